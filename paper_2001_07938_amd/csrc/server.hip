// Request server: continuous batching of SpMV and CG-solve requests over a
// pool of device-resident matrices.
//
// A scheduler thread runs "ticks".  Each tick admits waiting requests whose
// matrix is resident (while slots and the HBM budget allow), then issues ONE
// grouped product over every active request (y = A x for SpMV requests,
// q = A p for the next iteration of every active CG request) followed by
// three batched kernels that advance every CG by one iteration.  Requests
// that arrive while a tick runs join at the next tick; a CG request leaves
// after its last iteration, an SpMV request after its tick.  Uploads of
// matrices that are not resident run on a separate thread and stream, so
// they overlap with the ticks; least recently used idle matrices are evicted
// when the pool or the budget is full.  Every per-request reduction has a
// shape fixed by that request's matrix (its own tile list, its own number of
// CG workgroups), so a result does not depend on what else is in the batch.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <thread>
#include <unordered_map>
#include <vector>

#include "lilac_internal.h"

namespace lilac {
namespace {

using Clock = std::chrono::steady_clock;

int64_t now_ns()
{
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               Clock::now().time_since_epoch())
        .count();
}

struct SMatrix {
    int rows = 0, cols = 0;
    int64_t nnz = 0;
    const int32_t *rp = nullptr, *col = nullptr;
    const double *vals = nullptr;
    CsrHandle *h = nullptr;
    enum State { OFF, UPLOADING, READY } st = OFF;
    int64_t bytes = 0;         // device bytes while resident
    uint64_t last_use = 0;
    int refs = 0;              // admitted requests using it
    double *vin = nullptr, *vout = nullptr;  // trace-mode vectors
    int64_t spmv_bytes = 0;    // credited bytes of one product
    void *pin = nullptr;       // pinned host copy holding rp, col, vals
};

// Per-slot device workspace of an admitted request.
struct Slot {
    int64_t cap_n = 0, cap_chunks = 0;
    double *r = nullptr, *p = nullptr, *q = nullptr;
    double *pq = nullptr, *rr = nullptr;  // kBlock and 2*kBlock partials
    int32_t *done = nullptr;
    double *chunk = nullptr;
    int64_t bytes = 0;
};

struct Req {
    uint64_t ticket = 0;
    int kind = 0, mid = 0, iters = 0;
    const double *in = nullptr;
    double *out = nullptr;
    int64_t t_arr = 0;
    int iter = 0;          // CG iterations already enqueued
    int slot = -1;
    bool failed = false;
};

struct Tick {
    hipEvent_t ev = nullptr;
    std::vector<Req *> finishing;   // requests whose last work is in it
    bool pending = false;
    // pinned staging and device copies of the tick's tables
    char *host = nullptr, *dev = nullptr;
    size_t cap = 0;
};

struct Server {
    lilac_server_config cfg;
    hipStream_t stream = nullptr, up_stream = nullptr;
    std::vector<SMatrix> mats;
    // client side
    std::mutex mu;
    std::condition_variable cv, done_cv;
    std::deque<Req *> incoming;
    std::unordered_map<uint64_t, int> status;  // 0 pending, 1 done, -1 failed
    uint64_t next_ticket = 1;
    // scheduler side
    std::thread sched, uploader;
    std::atomic<bool> stop{false};
    std::deque<Req *> waiting;
    std::vector<Req *> active;
    std::vector<Slot> slots;
    std::vector<int> free_slots;
    int64_t used = 0, peak = 0;
    uint64_t use_clock = 0;
    int resident = 0;
    Tick ticks[2];
    int tick_no = 0;
    bool fifo = false;
    // uploads
    std::mutex up_mu;
    std::condition_variable up_cv;
    std::deque<int> up_q;
    std::vector<std::pair<int, CsrHandle *>> up_done;
    std::vector<int> up_failed;
    // statistics (under mu)
    std::vector<double> lat_us;
    int64_t n_spmv = 0, n_cg = 0, n_failed = 0, n_uploads = 0, n_evict = 0,
            n_ticks = 0;
    double bytes_done = 0.0;
    int64_t t_first = 0, t_last = 0;
    std::string err;
    int max_rows = 0;
    bool dead = false;   // the scheduler stopped on an error
};

int64_t matrix_bytes(const SMatrix &m)
{
    const int64_t npad = ((m.nnz + kPad - 1) / kPad) * kPad + kPad;
    return (int64_t)(m.rows + 1) * 4 + npad * 12 + (int64_t)m.rows * 4 +
           (int64_t)(m.rows + m.cols) * 8 + (1 << 20);
}

void free_slot_mem(Slot &sl)
{
    dev_free(sl.r);
    dev_free(sl.p);
    dev_free(sl.q);
    dev_free(sl.pq);
    dev_free(sl.rr);
    dev_free(sl.done);
    dev_free(sl.chunk);
    sl = Slot();
}

// ------------------------------------------------------------- uploads

void upload_loop(Server *S)
{
    if (hipSetDevice(lib_device()) != hipSuccess)
        return;
    while (!S->stop.load()) {
        int id = -1;
        {
            std::unique_lock<std::mutex> lk(S->up_mu);
            S->up_cv.wait_for(lk, std::chrono::milliseconds(5),
                              [&] { return !S->up_q.empty() || S->stop.load(); });
            if (S->stop.load())
                return;
            if (S->up_q.empty())
                continue;
            id = S->up_q.front();
            S->up_q.pop_front();
        }
        SMatrix &m = S->mats[id];
        CsrHandle *h = nullptr;
        // the arrays go up from pinned host memory into staging buffers
        // without the library lock (the scheduler may need it meanwhile, to
        // evict); the lock is taken only to build the handle from them
        int32_t *d_rp = nullptr, *d_col = nullptr;
        double *d_vals = nullptr;
        const size_t b_rp = (size_t)(m.rows + 1) * 4, b_col = (size_t)m.nnz * 4,
                     b_vals = (size_t)m.nnz * 8;
        try {
            {
                std::lock_guard<std::recursive_mutex> lk(lib_mutex());
                d_rp = (int32_t *)dev_alloc(b_rp);
                d_col = (int32_t *)dev_alloc(std::max<size_t>(b_col, 4));
                d_vals = (double *)dev_alloc(std::max<size_t>(b_vals, 8));
            }
            HIPC(hipMemcpyAsync(d_rp, m.rp, b_rp, hipMemcpyHostToDevice, S->up_stream));
            if (m.nnz) {
                HIPC(hipMemcpyAsync(d_col, m.col, b_col, hipMemcpyHostToDevice, S->up_stream));
                HIPC(hipMemcpyAsync(d_vals, m.vals, b_vals, hipMemcpyHostToDevice,
                                    S->up_stream));
            }
            HIPC(hipStreamSynchronize(S->up_stream));
            std::lock_guard<std::recursive_mutex> lk(lib_mutex());
            h = create_handle(m.rows, m.cols, m.nnz, d_rp, d_col, d_vals, LILAC_F64, 0,
                              true);
            dev_free(d_rp);
            dev_free(d_col);
            dev_free(d_vals);
            d_rp = d_col = nullptr;
            d_vals = nullptr;
            m.vin = (double *)dev_alloc((size_t)std::max(1, m.cols) * 8);
            m.vout = (double *)dev_alloc((size_t)std::max(1, m.rows) * 8);
            // trace-mode operands: x (or b) = 1
            std::vector<double> ones((size_t)std::max(1, m.cols), 1.0);
            HIPC(hipMemcpyAsync(m.vin, ones.data(), ones.size() * 8,
                                hipMemcpyHostToDevice, S->up_stream));
            HIPC(hipStreamSynchronize(S->up_stream));
        } catch (const Error &e) {
            {
                std::lock_guard<std::recursive_mutex> lk(lib_mutex());
                dev_free(d_rp);
                dev_free(d_col);
                dev_free(d_vals);
            }
            std::lock_guard<std::mutex> lk(S->up_mu);
            S->up_failed.push_back(id);
            S->err = e.msg;
            continue;
        }
        std::lock_guard<std::mutex> lk(S->up_mu);
        S->up_done.emplace_back(id, h);
    }
}

// ------------------------------------------------------------- scheduler

bool evict_one(Server *S)
{
    int best = -1;
    for (int i = 0; i < (int)S->mats.size(); ++i) {
        const SMatrix &m = S->mats[i];
        if (m.st == SMatrix::READY && m.refs == 0 &&
            (best < 0 || m.last_use < S->mats[best].last_use))
            best = i;
    }
    if (best < 0)
        return false;
    SMatrix &m = S->mats[best];
    {
        std::lock_guard<std::recursive_mutex> lk(lib_mutex());
        destroy_handle(m.h);
        dev_free(m.vin);
        dev_free(m.vout);
    }
    m.h = nullptr;
    m.vin = m.vout = nullptr;
    m.st = SMatrix::OFF;
    S->used -= m.bytes;
    m.bytes = 0;
    S->resident -= 1;
    S->n_evict += 1;
    return true;
}

void finish(Server *S, Req *r, int64_t t)
{
    SMatrix &m = S->mats[r->mid];
    m.refs -= 1;
    if (r->slot >= 0)
        S->free_slots.push_back(r->slot);
    std::lock_guard<std::mutex> lk(S->mu);
    if (r->failed) {
        S->status[r->ticket] = -1;
        S->n_failed += 1;
    } else {
        S->status[r->ticket] = 1;
        S->lat_us.push_back((t - r->t_arr) * 1e-3);
        if (r->kind == LILAC_REQ_CG) {
            S->n_cg += 1;
            S->bytes_done += (double)r->iters * (m.spmv_bytes + 9.0 * m.rows * 8);
        } else {
            S->n_spmv += 1;
            S->bytes_done += (double)m.spmv_bytes;
        }
        if (!S->t_first)
            S->t_first = r->t_arr;
        S->t_last = std::max(S->t_last, t);
    }
    S->done_cv.notify_all();
    delete r;
}

void complete_tick(Server *S, Tick &tk)
{
    if (!tk.pending)
        return;
    HIPC(hipEventSynchronize(tk.ev));
    const int64_t t = now_ns();
    for (Req *r : tk.finishing)
        finish(S, r, t);
    tk.finishing.clear();
    tk.pending = false;
}

// A workspace slot for request r.  Slots are sized for the largest
// registered matrix, so any free slot fits; chunk partials grow on demand.
bool get_slot(Server *S, Req *r)
{
    const SMatrix &m = S->mats[r->mid];
    const int64_t nc = m.h->nchunks;
    if (S->free_slots.empty()) {
        if ((int)S->slots.size() >= S->cfg.max_active)
            return false;
        const int64_t n = S->max_rows;
        const int64_t need = n * 24 + 3 * kBlock * 8 + 256 + 4096;
        if (S->used + need > S->cfg.hbm_budget)
            return false;
        Slot sl;
        std::lock_guard<std::recursive_mutex> lk(lib_mutex());
        sl.cap_n = n;
        sl.r = (double *)dev_alloc((size_t)std::max<int64_t>(n, 1) * 8);
        sl.p = (double *)dev_alloc((size_t)std::max<int64_t>(n, 1) * 8);
        sl.q = (double *)dev_alloc((size_t)std::max<int64_t>(n, 1) * 8);
        sl.pq = (double *)dev_alloc(kBlock * 8);
        sl.rr = (double *)dev_alloc(2 * kBlock * 8);
        sl.done = (int32_t *)dev_alloc(256);
        sl.bytes = need;
        S->used += need;
        S->peak = std::max(S->peak, S->used);
        S->slots.push_back(sl);
        S->free_slots.push_back((int)S->slots.size() - 1);
    }
    const int si = S->free_slots.back();
    Slot &sl = S->slots[si];
    if (sl.cap_chunks < nc) {
        if (S->used + nc * 8 > S->cfg.hbm_budget)
            return false;
        std::lock_guard<std::recursive_mutex> lk(lib_mutex());
        dev_free(sl.chunk);
        sl.chunk = (double *)dev_alloc((size_t)nc * 8);
        S->used += (nc - sl.cap_chunks) * 8;
        sl.bytes += (nc - sl.cap_chunks) * 8;
        sl.cap_chunks = nc;
        S->peak = std::max(S->peak, S->used);
    }
    r->slot = si;
    S->free_slots.pop_back();
    return true;
}

void collect_uploads(Server *S)
{
    std::vector<std::pair<int, CsrHandle *>> done;
    std::vector<int> failed;
    {
        std::lock_guard<std::mutex> lk(S->up_mu);
        done.swap(S->up_done);
        failed.swap(S->up_failed);
    }
    for (auto &d : done) {
        SMatrix &m = S->mats[d.first];
        m.h = d.second;
        m.st = SMatrix::READY;
        m.spmv_bytes = m.nnz * 12 + (int64_t)(m.rows + 1) * 4 +
                       (int64_t)(m.cols + m.rows) * 8;
    }
    for (int id : failed) {
        SMatrix &m = S->mats[id];
        m.st = SMatrix::OFF;
        S->used -= m.bytes;
        m.bytes = 0;
        S->resident -= 1;
        // fail every waiting request on this matrix
        for (auto it = S->waiting.begin(); it != S->waiting.end();) {
            if ((*it)->mid == id) {
                (*it)->failed = true;
                m.refs += 1;
                finish(S, *it, now_ns());
                it = S->waiting.erase(it);
            } else {
                ++it;
            }
        }
    }
}

// Start an upload if the budget and the pool allow (evicting idle matrices).
void request_upload(Server *S, int id)
{
    SMatrix &m = S->mats[id];
    const int64_t need = matrix_bytes(m);
    if (need > S->cfg.hbm_budget) {
        m.st = SMatrix::UPLOADING;   // will fail through the failure path
        S->used += 0;
        std::lock_guard<std::mutex> lk(S->up_mu);
        S->up_failed.push_back(id);
        S->err = "matrix larger than the server's HBM budget";
        S->resident += 1;
        return;
    }
    while ((S->used + need > S->cfg.hbm_budget ||
            S->resident >= S->cfg.pool_capacity) &&
           evict_one(S)) {
    }
    if (S->used + need > S->cfg.hbm_budget || S->resident >= S->cfg.pool_capacity)
        return;  // try again when something becomes idle
    m.st = SMatrix::UPLOADING;
    m.bytes = need;
    S->used += need;
    S->peak = std::max(S->peak, S->used);
    S->resident += 1;
    S->n_uploads += 1;
    std::lock_guard<std::mutex> lk(S->up_mu);
    S->up_q.push_back(id);
    S->up_cv.notify_one();
}

// Grows the pinned and device table buffers of a tick.
void tick_reserve(Tick &tk, size_t bytes)
{
    if (bytes <= tk.cap)
        return;
    size_t cap = std::max<size_t>(bytes, 2 * tk.cap);
    cap = std::max<size_t>(cap, 1 << 16);
    if (tk.host)
        (void)hipHostFree(tk.host);
    if (tk.dev) {
        std::lock_guard<std::recursive_mutex> lk(lib_mutex());
        dev_free(tk.dev);
    }
    HIPC(hipHostMalloc((void **)&tk.host, cap, hipHostMallocDefault));
    {
        std::lock_guard<std::recursive_mutex> lk(lib_mutex());
        tk.dev = (char *)dev_alloc(cap);
    }
    tk.cap = cap;
}

// One batched tick over every active request.
void run_tick(Server *S)
{
    Tick &tk = S->ticks[S->tick_no & 1];
    complete_tick(S, tk);  // its buffers are about to be reused
    std::vector<MatDesc> descs;
    std::vector<int32_t> prefix(1, 0);
    std::vector<int32_t> items;
    std::vector<CgSeg> init, step;
    std::vector<Req *> own;
    int32_t init_blocks = 0, step_blocks = 0;
    for (Req *r : S->active) {
        SMatrix &m = S->mats[r->mid];
        Slot &sl = S->slots[r->slot];
        const int j = (int)descs.size();
        const double *in = r->in ? r->in : m.vin;
        double *out = r->out ? r->out : m.vout;
        if (own_layout(*m.h)) {
            // matrices in a layout of their own run their own product kernel
            own.push_back(r);
        } else if (r->kind == LILAC_REQ_SPMV) {
            descs.push_back(make_desc(*m.h, in, out, nullptr, sl.chunk));
        } else {
            descs.push_back(make_desc(*m.h, sl.p, sl.q, nullptr, sl.chunk));
        }
        if (r->kind == LILAC_REQ_CG) {
            CgSeg sg;
            sg.b = in;
            sg.x = out;
            sg.r = sl.r;
            sg.p = sl.p;
            sg.q = sl.q;
            sg.pq_part = sl.pq;
            sg.rr_part = sl.rr;
            sg.done = sl.done;
            sg.n = m.rows;
            sg.nb = cg_seg_blocks(m.rows);
            sg.iter = r->iter;
            sg.pad = 0;
            if (r->iter == 0) {
                sg.blk0 = init_blocks;
                init_blocks += sg.nb;
                init.push_back(sg);
            }
            sg.blk0 = step_blocks;
            step_blocks += sg.nb;
            step.push_back(sg);
        }
        if (own_layout(*m.h))
            continue;
        prefix.push_back(prefix.back() + m.h->ntiles);
        for (int32_t k = 0; k < m.h->nsplit; ++k) {
            items.push_back(j);
            items.push_back(k);
        }
    }
    // column-panel products of the tick: one grouped launch
    std::vector<PanelDesc> pdesc;
    std::vector<PanelIO> pio;
    std::vector<int32_t> pprefix(1, 0);
    std::vector<BandDesc> bdesc;
    std::vector<PanelIO> bio;
    std::vector<int32_t> bprefix(1, 0);
    std::vector<Req *> own_hot;
    // matrices with the most non-zeros per block first, so that a grouped
    // launch ends on short blocks
    std::vector<Req *> heavy(own.begin(), own.end());
    auto per_block = [&](const Req *r) {
        const CsrHandle &h = *S->mats[r->mid].h;
        const int32_t nb = h.use_panels ? h.pan.nblk : h.use_band ? h.band.nblk : 1;
        return (double)h.nnz / (double)std::max(1, nb);
    };
    std::stable_sort(heavy.begin(), heavy.end(),
                     [&](const Req *a, const Req *b) { return per_block(a) > per_block(b); });
    for (Req *r : heavy) {
        SMatrix &m = S->mats[r->mid];
        Slot &sl = S->slots[r->slot];
        const PanelIO io = (r->kind == LILAC_REQ_SPMV)
                               ? PanelIO{r->in ? r->in : m.vin, r->out ? r->out : m.vout}
                               : PanelIO{sl.p, sl.q};
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
    const size_t b_items = ((items.size() * 4 + 15) / 16) * 16;
    const size_t b_init = init.size() * sizeof(CgSeg);
    const size_t b_step = step.size() * sizeof(CgSeg);
    const size_t b_pdesc = pdesc.size() * sizeof(PanelDesc);
    const size_t b_pio = pio.size() * sizeof(PanelIO);
    const size_t b_ppre = ((pprefix.size() * 4 + 15) / 16) * 16;
    const size_t b_bdesc = bdesc.size() * sizeof(BandDesc);
    const size_t b_bio = bio.size() * sizeof(PanelIO);
    const size_t b_bpre = ((bprefix.size() * 4 + 15) / 16) * 16;
    tick_reserve(tk, b_desc + b_pre + b_items + b_init + b_step + b_pdesc + b_pio +
                         b_ppre + b_bdesc + b_bio + b_bpre + 64);
    size_t off = 0;
    auto put = [&](const void *src, size_t n, size_t padded) {
        std::memcpy(tk.host + off, src, n);
        const size_t at = off;
        off += padded;
        return at;
    };
    const size_t o_desc = put(descs.data(), b_desc, b_desc);
    const size_t o_pre = put(prefix.data(), prefix.size() * 4, b_pre);
    const size_t o_items = put(items.data(), items.size() * 4, b_items);
    const size_t o_init = put(init.data(), b_init, b_init);
    const size_t o_step = put(step.data(), b_step, b_step);
    const size_t o_pdesc = put(pdesc.data(), b_pdesc, b_pdesc);
    const size_t o_pio = put(pio.data(), b_pio, b_pio);
    const size_t o_ppre = put(pprefix.data(), pprefix.size() * 4, b_ppre);
    const size_t o_bdesc = put(bdesc.data(), b_bdesc, b_bdesc);
    const size_t o_bio = put(bio.data(), b_bio, b_bio);
    const size_t o_bpre = put(bprefix.data(), bprefix.size() * 4, b_bpre);
    HIPC(hipMemcpyAsync(tk.dev, tk.host, off, hipMemcpyHostToDevice, S->stream));
    const MatDesc *d_desc = (const MatDesc *)(tk.dev + o_desc);
    if (!init.empty())
        launch_cgb_init((const CgSeg *)(tk.dev + o_init), (int32_t)init.size(),
                        init_blocks, S->stream);
    launch_spmv_segments(LILAC_F64, d_desc, (const int32_t *)(tk.dev + o_pre),
                         (int32_t)descs.size(), prefix.back(), tile_grid(LILAC_F64),
                         S->stream);
    launch_spmv_panels_grouped(LILAC_F64, (const PanelDesc *)(tk.dev + o_pdesc),
                               (const PanelIO *)(tk.dev + o_pio),
                               (const int32_t *)(tk.dev + o_ppre), (int32_t)pdesc.size(),
                               pprefix.back(), S->stream);
    launch_spmv_band_grouped(LILAC_F64, (const BandDesc *)(tk.dev + o_bdesc),
                             (const PanelIO *)(tk.dev + o_bio),
                             (const int32_t *)(tk.dev + o_bpre), (int32_t)bdesc.size(),
                             bprefix.back(), S->stream);
    for (Req *r : own_hot) {
        SMatrix &m = S->mats[r->mid];
        Slot &sl = S->slots[r->slot];
        if (r->kind == LILAC_REQ_SPMV)
            spmv_enqueue(*m.h, r->in ? r->in : m.vin, r->out ? r->out : m.vout,
                         Epi{EPI_NONE, 0, 0.0, 0.0}, nullptr, false, S->stream);
        else
            spmv_enqueue(*m.h, sl.p, sl.q, Epi{EPI_NONE, 0, 0.0, 0.0}, nullptr,
                         false, S->stream);
    }
    if (!items.empty()) {
        MatDesc none{};
        launch_split_finalize(LILAC_F64, (const int32_t *)(tk.dev + o_items),
                              (int32_t)(items.size() / 2), none, d_desc,
                              Epi{EPI_NONE, 0, 0.0, 0.0}, nullptr, S->stream);
    }
    if (!step.empty()) {
        const CgSeg *d_step = (const CgSeg *)(tk.dev + o_step);
        launch_cgb_pq(d_step, (int32_t)step.size(), step_blocks, S->stream);
        launch_cgb_update(d_step, (int32_t)step.size(), step_blocks, S->stream);
        launch_cgb_xpay(d_step, (int32_t)step.size(), step_blocks, S->stream);
    }
    HIPC(hipEventRecord(tk.ev, S->stream));
    tk.pending = true;
    S->n_ticks += 1;
    // requests whose last step is in this tick leave the active set now;
    // their resources are released when the tick completes
    std::vector<Req *> still;
    for (Req *r : S->active) {
        if (r->kind == LILAC_REQ_CG) {
            r->iter += 1;
            if (r->iter < r->iters) {
                still.push_back(r);
                continue;
            }
        }
        tk.finishing.push_back(r);
    }
    S->active.swap(still);
    S->tick_no += 1;
}

// The plain path: one request at a time with the single-matrix calls.
void run_fifo_one(Server *S, Req *r)
{
    SMatrix &m = S->mats[r->mid];
    const double *in = r->in ? r->in : m.vin;
    double *out = r->out ? r->out : m.vout;
    if (r->kind == LILAC_REQ_SPMV) {
        spmv_enqueue(*m.h, in, out, Epi{EPI_NONE, 0, 0.0, 0.0}, nullptr,
                     false, S->stream);
    } else {
        std::lock_guard<std::recursive_mutex> lk(lib_mutex());
        run_cg(*m.h, in, out, r->iters, LILAC_CG_GRAPH, S->stream, nullptr,
               nullptr);
    }
    HIPC(hipStreamSynchronize(S->stream));
    finish(S, r, now_ns());
}

void schedule_loop(Server *S)
{
    HIPC(hipSetDevice(lib_device()));
    while (true) {
        {
            std::unique_lock<std::mutex> lk(S->mu);
            while (!S->incoming.empty()) {
                S->waiting.push_back(S->incoming.front());
                S->incoming.pop_front();
            }
        }
        collect_uploads(S);
        if (S->stop.load()) {
            // shutting down: what has not started fails, what runs finishes
            for (Req *r : S->waiting) {
                r->failed = true;
                S->mats[r->mid].refs += 1;
                finish(S, r, now_ns());
            }
            S->waiting.clear();
            if (S->active.empty()) {
                complete_tick(S, S->ticks[0]);
                complete_tick(S, S->ticks[1]);
                break;
            }
        }
        // admission, in arrival order; a request whose matrix is not yet
        // resident does not hold up the ones behind it
        for (auto it = S->waiting.begin(); it != S->waiting.end();) {
            Req *r = *it;
            SMatrix &m = S->mats[r->mid];
            if (m.st == SMatrix::OFF) {
                request_upload(S, r->mid);
                ++it;
                continue;
            }
            if (m.st != SMatrix::READY) {
                ++it;
                continue;
            }
            if (S->fifo) {
                it = S->waiting.erase(it);
                m.refs += 1;
                m.last_use = ++S->use_clock;
                run_fifo_one(S, r);
                break;
            }
            if ((int)S->active.size() >= S->cfg.max_active)
                break;
            m.refs += 1;  // keep it resident while we look for a slot
            if (!get_slot(S, r)) {
                m.refs -= 1;
                break;
            }
            m.last_use = ++S->use_clock;
            S->active.push_back(r);
            it = S->waiting.erase(it);
        }
        if (!S->active.empty()) {
            run_tick(S);
            // keep one tick in flight: finish the previous one now
            complete_tick(S, S->ticks[S->tick_no & 1]);
            continue;
        }
        complete_tick(S, S->ticks[0]);
        complete_tick(S, S->ticks[1]);
        std::unique_lock<std::mutex> lk(S->mu);
        S->cv.wait_for(lk, std::chrono::microseconds(200),
                       [&] { return !S->incoming.empty() || S->stop.load(); });
    }
}

void scheduler_main(Server *S)
{
    try {
        schedule_loop(S);
    } catch (const Error &e) {
        std::lock_guard<std::mutex> lk(S->mu);
        S->err = e.msg;
        S->dead = true;
        // fail everything still queued so waiters return
        for (Req *r : S->waiting)
            S->status[r->ticket] = -1;
        for (Req *r : S->active)
            S->status[r->ticket] = -1;
        for (Req *r : S->incoming)
            S->status[r->ticket] = -1;
        S->done_cv.notify_all();
    }
}

void fill_stats(Server *S, lilac_server_stats *o)
{
    std::lock_guard<std::mutex> lk(S->mu);
    std::memset(o, 0, sizeof(*o));
    o->completed = (int64_t)S->lat_us.size();
    o->spmv_done = S->n_spmv;
    o->cg_done = S->n_cg;
    o->failed = S->n_failed;
    o->uploads = S->n_uploads;
    o->evictions = S->n_evict;
    o->ticks = S->n_ticks;
    o->peak_device_bytes = S->peak;
    if (!S->lat_us.empty()) {
        std::vector<double> v = S->lat_us;
        auto pct = [&](double p) {
            const size_t k = std::min(v.size() - 1, (size_t)(p * (v.size() - 1) + 0.5));
            std::nth_element(v.begin(), v.begin() + k, v.end());
            return v[k];
        };
        o->p50_us = pct(0.50);
        o->p99_us = pct(0.99);
        double s = 0.0, mx = 0.0;
        for (double x : S->lat_us) {
            s += x;
            mx = std::max(mx, x);
        }
        o->mean_us = s / (double)S->lat_us.size();
        o->max_us = mx;
    }
    const double wall = (S->t_last - S->t_first) * 1e-9;
    o->wall_s = wall;
    if (wall > 0) {
        o->req_per_s = o->completed / wall;
        o->solves_per_s = S->n_cg / wall;
        o->gbytes_per_s = S->bytes_done / wall / 1e9;
    }
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
        S->cfg.pool_capacity = (cfg && cfg->pool_capacity > 0) ? cfg->pool_capacity : 64;
        S->cfg.fifo = cfg ? cfg->fifo : 0;
        S->fifo = S->cfg.fifo != 0;
        HIPC(hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking));
        HIPC(hipStreamCreateWithFlags(&S->up_stream, hipStreamNonBlocking));
        for (auto &t : S->ticks)
            HIPC(hipEventCreateWithFlags(&t.ev, hipEventDisableTiming));
        S->sched = std::thread(scheduler_main, S);
        S->uploader = std::thread(upload_loop, S);
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
        std::lock_guard<std::mutex> lk(S->mu);
        if (!S->waiting.empty() || !S->active.empty() || !S->incoming.empty())
            fail(LILAC_ERR_STATE, "add matrices before submitting requests");
        SMatrix m;
        m.rows = rows;
        m.cols = cols >= 0 ? cols : rows;
        m.nnz = nnz;
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
        if (r->kind == LILAC_REQ_CG && (r->iters <= 0 ||
                                        S->mats[r->matrix].rows != S->mats[r->matrix].cols))
            fail(LILAC_ERR_ARG, "CG needs iters > 0 and a square matrix");
        {
            std::lock_guard<std::mutex> lk(S->mu);
            if (S->dead)
                fail(LILAC_ERR_STATE, "server stopped after an error: " + S->err);
        }
        auto *q = new Req();
        q->kind = r->kind;
        q->mid = r->matrix;
        q->iters = r->iters;
        q->in = r->in;
        q->out = r->out;
        q->t_arr = r->arrival_ns > 0 ? r->arrival_ns : now_ns();
        std::lock_guard<std::mutex> lk(S->mu);
        q->ticket = S->next_ticket++;
        S->status[q->ticket] = 0;
        S->incoming.push_back(q);
        S->cv.notify_one();
        if (ticket)
            *ticket = q->ticket;
    });
}

int lilac_server_poll(lilac_server_t hs, uint64_t ticket, int *done)
{
    Server *S = (Server *)hs;
    return sguard([&] {
        if (!S || !done)
            fail(LILAC_ERR_ARG, "bad argument");
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->status.find(ticket);
        if (it == S->status.end())
            fail(LILAC_ERR_ARG, "unknown ticket");
        *done = it->second;
    });
}

int lilac_server_wait(lilac_server_t hs, uint64_t ticket)
{
    Server *S = (Server *)hs;
    return sguard([&] {
        if (!S)
            fail(LILAC_ERR_ARG, "bad argument");
        std::unique_lock<std::mutex> lk(S->mu);
        auto it = S->status.find(ticket);
        if (it == S->status.end())
            fail(LILAC_ERR_ARG, "unknown ticket");
        S->done_cv.wait(lk, [&] { return S->status[ticket] != 0; });
        if (S->status[ticket] < 0)
            fail(LILAC_ERR_STATE, "request failed: " + S->err);
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
        fill_stats(S, out);
    });
}

int lilac_server_reset_stats(lilac_server_t hs)
{
    Server *S = (Server *)hs;
    return sguard([&] {
        if (!S)
            fail(LILAC_ERR_ARG, "bad argument");
        std::lock_guard<std::mutex> lk(S->mu);
        S->lat_us.clear();
        S->n_spmv = S->n_cg = S->n_failed = S->n_uploads = S->n_evict = S->n_ticks = 0;
        S->bytes_done = 0.0;
        S->t_first = S->t_last = 0;
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
                (kind[i] != LILAC_REQ_SPMV && kind[i] != LILAC_REQ_CG))
                fail(LILAC_ERR_ARG, "bad request in trace");
        lilac_server_reset_stats(hs);
        std::vector<uint64_t> tickets((size_t)n);
        const int64_t t0 = now_ns() + 1000000;  // start 1 ms from now
        for (int i = 0; i < n; ++i) {
            const int64_t due = t0 + arrival_ns[i];
            int64_t t = now_ns();
            if (due - t > 200000)
                std::this_thread::sleep_for(std::chrono::nanoseconds(due - t - 100000));
            while ((t = now_ns()) < due) {
            }
            auto *q = new Req();
            q->kind = kind[i];
            q->mid = matrix[i];
            q->iters = cg_iters;
            q->t_arr = due;
            // trace mode: the matrix's own vectors (attached at admission)
            q->in = nullptr;
            q->out = nullptr;
            std::lock_guard<std::mutex> lk(S->mu);
            q->ticket = S->next_ticket++;
            S->status[q->ticket] = 0;
            S->incoming.push_back(q);
            tickets[(size_t)i] = q->ticket;
            S->cv.notify_one();
        }
        {
            std::unique_lock<std::mutex> lk(S->mu);
            for (uint64_t tkt : tickets)
                S->done_cv.wait(lk, [&] { return S->status[tkt] != 0; });
            for (uint64_t tkt : tickets)
                S->status.erase(tkt);
        }
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
        S->cv.notify_all();
        S->up_cv.notify_all();
        if (S->sched.joinable())
            S->sched.join();
        if (S->uploader.joinable())
            S->uploader.join();
        (void)hipStreamSynchronize(S->stream);
        std::lock_guard<std::recursive_mutex> lk(lib_mutex());
        for (auto &d : S->up_done)   // uploads that finished after the stop
            destroy_handle(d.second);
        for (auto &m : S->mats) {
            if (m.h)
                destroy_handle(m.h);
            dev_free(m.vin);
            dev_free(m.vout);
            if (m.pin)
                (void)hipHostFree(m.pin);
        }
        for (auto &sl : S->slots)
            free_slot_mem(sl);
        for (auto &t : S->ticks) {
            if (t.host)
                (void)hipHostFree(t.host);
            dev_free(t.dev);
            (void)hipEventDestroy(t.ev);
        }
        for (auto *r : S->waiting)
            delete r;
        for (auto *r : S->incoming)
            delete r;
        (void)hipStreamDestroy(S->stream);
        (void)hipStreamDestroy(S->up_stream);
        delete S;
    });
}

}  // extern "C"

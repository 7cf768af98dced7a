// Scheduling core of the request server: admission against an HBM byte
// budget, a bounded pool of resident matrices with eviction, request slots,
// continuous batching into ticks, completion and latency statistics.
//
// Nothing here touches the device.  Every device action (upload, eviction,
// slot memory, launching and waiting for a tick, the one-request-at-a-time
// path) is a call on an Executor, so the same scheduling code runs in the
// library, where the Executor drives HIP, and on the CPU under a simulated
// executor with virtual time (and under the sanitizers) in the tests.
//
// This is the paper's persistent-state marshaling (section "LiLAC-How",
// paragraphs "Persistence" and "Data Marshaling": a matrix is copied to the
// device once and reused until it has to go) applied to a stream of
// independent requests instead of one program's call sites.
//
// Requests run in two lanes, each with its own ticks (on its own device
// stream in the library): matrices whose one product is long go to the
// heavy lane, the rest to the light lane, so that a short request never
// waits out the long product of another request's tick.
//
// Threads: one scheduler thread calls step(); any thread may call submit,
// poll, wait, stats; executor threads report finished uploads through
// upload_done.  Scheduler-only state is touched by step() alone.
#pragma once

#include <condition_variable>
#include <cstdint>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <atomic>
#include <vector>

namespace lilac {
namespace serve {

constexpr int kSpmv = 0;
constexpr int kCg = 1;
constexpr int kLanes = 2;   // 0: light, 1: heavy

struct Request {
    uint64_t ticket = 0;
    int kind = kSpmv;
    int mid = 0;                // matrix id
    int iters = 0;              // CG iterations
    const void *in = nullptr;   // device x (SpMV) or b (CG); null: the server's own
    void *out = nullptr;        // device y (SpMV) or x (CG); null: the slot's own
    int64_t t_arr = 0;          // arrival, executor clock (ns)
    int64_t t_adm = 0;          // admission (set by the core)
    int iter = 0;               // CG iterations launched so far
    int slot = -1;
    bool failed = false;
};

struct Limits {
    int64_t budget = 0;        // device bytes for matrices, slots and overhead
    int max_active = 1;        // requests admitted at once
    int pool_capacity = 1;     // matrices resident or uploading at once
    bool fifo = false;         // one request at a time, no batching
    int64_t overhead = 0;      // bytes set aside for the server's own buffers
};

struct Stats {
    int64_t completed = 0, spmv_done = 0, cg_done = 0, failed = 0;
    double p50_us = 0, p99_us = 0, mean_us = 0, max_us = 0;
    double wall_s = 0, req_per_s = 0, solves_per_s = 0, gbytes_per_s = 0;
    int64_t uploads = 0, evictions = 0, ticks = 0;
    int64_t planned_peak = 0;  // highest planned device bytes (charges + reserves)
    double mean_wait_us = 0;   // arrival -> admission (upload, slot, queue)
    double mean_run_us = 0;    // admission -> completion
    int64_t waited_upload = 0; // requests that found their matrix not resident
};

class Executor {
  public:
    virtual ~Executor() = default;
    virtual int64_t now_ns() = 0;
    // Bytes to set aside before matrix `mid` is uploaded: a bound on what
    // the upload and the build of its resident copy hold at any moment.
    virtual int64_t upload_reserve(int mid) = 0;
    // Starts the upload; its end is reported through Core::upload_done.
    virtual void start_upload(int mid) = 0;
    // Gives up the resident copy of `mid` (no request uses it).  The memory
    // may come back later, but before any upload or slot allocation after
    // this call takes device memory.
    virtual void evict(int mid) = 0;
    // Total device bytes slot `slot` must hold to serve a request on `mid`.
    virtual int64_t slot_need(int slot, int mid) = 0;
    // Allocates or grows slot `slot` to that size.  Blocking.
    virtual void prepare_slot(int slot, int mid) = 0;
    // Frees an unused slot's memory.  Blocking.
    virtual void release_slot(int slot) = 0;
    // Lane of a matrix's requests (0 light, 1 heavy).
    virtual int lane_of(int mid) = 0;
    // Enqueues one batched step of a lane over `reqs`: the product of every
    // SpMV request and one iteration of every CG request (iteration
    // r->iter).  A lane has two tick buffers (tick 0 and 1), used in turn.
    virtual void launch_tick(int lane, int tick, const std::vector<Request *> &reqs) = 0;
    // Whether a launched tick has finished on the device (non-blocking).
    virtual bool tick_done(int lane, int tick) = 0;
    // Blocks until it has.
    virtual void wait_tick(int lane, int tick) = 0;
    // The plain path: runs the whole request alone.  Blocking.
    virtual void run_one(Request *r) = 0;
};

class Core {
  public:
    Core(Executor &ex, const Limits &lim);
    ~Core();
    Core(const Core &) = delete;
    Core &operator=(const Core &) = delete;

    // Registers a matrix (before the first request): the credited bytes of
    // one product and of one CG iteration, for the throughput figures.
    int add_matrix(int64_t spmv_bytes, int64_t cg_iter_bytes);
    int matrix_count() const { return (int)mats_.size(); }

    // ---- client side (any thread) ----
    uint64_t submit(Request *r);   // takes ownership
    int poll(uint64_t ticket);     // 0 pending, 1 done, -1 failed, -2 unknown
    int wait(uint64_t ticket);     // blocks; 1 done, -1 failed, -2 unknown
    void forget(uint64_t ticket);  // drops a finished ticket's status
    Stats stats();
    void reset_stats();
    std::string error();
    bool dead();

    // ---- executor side (any thread) ----
    void upload_done(int mid, bool ok, int64_t held_bytes, const std::string &err);

    // ---- scheduler thread ----
    // One scheduling round: take new requests and finished uploads, admit,
    // finish the ticks that are done, launch a tick in every lane that has
    // active requests and a free tick buffer.  Returns false when there was
    // nothing to do.
    bool step();
    // Whether a tick is still running (the scheduler should poll again soon).
    bool busy() const;
    // Waits (real time) until a request or an upload result arrives.
    void wait_for_work(int64_t max_ns);
    // Wakes a scheduler blocked in wait_for_work.
    void wake();
    // Fails what has not started, finishes what runs.
    void shutdown();
    // Marks the server failed after an executor error: every outstanding
    // request fails and later submits are refused.
    void die(const std::string &msg);

    // ---- observation (scheduler thread, or after it stopped) ----
    int64_t planned_bytes() const { return charged_; }
    int64_t planned_peak() const { return peak_; }
    int resident() const { return resident_; }
    int active() const { return (int)(active_[0].size() + active_[1].size()); }
    int waiting() const { return (int)waiting_.size(); }
    int uploading() const;
    bool is_resident(int mid) const;
    bool is_ready(int mid) const;
    int64_t matrix_charge(int mid) const { return mats_[(size_t)mid].charge; }
    int64_t reserve_overruns() const { return overruns_; }

  private:
    enum MState { OFF, UPLOADING, READY };
    struct Mat {
        MState st = OFF;
        int64_t charge = 0;      // planned bytes while resident or uploading
        int refs = 0;            // admitted requests using it
        int queued = 0;          // waiting requests naming it
        uint64_t last_use = 0;   // admission clock of the last two uses
        uint64_t prev_use = 0;
        int64_t spmv_bytes = 0, cg_iter_bytes = 0;
    };
    struct Slot {
        int64_t charge = 0;
        bool busy = false;
    };
    struct Done {
        int mid;
        bool ok;
        int64_t held;
        std::string err;
    };

    bool try_upload(int mid);
    int pick_victim() const;
    bool make_room(int64_t need, bool for_upload);
    void evict(int mid);
    bool get_slot(Request *r);
    void finish(Request *r, int64_t t);
    void fail_waiting_on(int mid, const std::string &why);
    bool launch(int lane);
    void complete(int lane, int tick);
    void collect_uploads();
    void take_incoming();
    void bump_peak();

    Executor &ex_;
    Limits lim_;
    std::vector<Mat> mats_;
    std::vector<Slot> slots_;
    std::vector<int> free_slots_;
    std::deque<Request *> waiting_;
    std::vector<Request *> active_[kLanes];
    std::vector<Request *> finishing_[kLanes][2];
    bool pending_[kLanes][2] = {{false, false}, {false, false}};
    int tick_no_[kLanes] = {0, 0};
    int64_t charged_ = 0, peak_ = 0;
    int resident_ = 0;
    uint64_t use_clock_ = 0;
    int64_t overruns_ = 0;

    // client side, under mu_
    std::mutex mu_;
    std::condition_variable work_cv_, done_cv_;
    std::deque<Request *> incoming_;
    std::unordered_map<uint64_t, int> status_;
    uint64_t next_ticket_ = 1;
    std::vector<double> lat_us_;
    double wait_sum_us_ = 0.0, run_sum_us_ = 0.0;
    int64_t n_waited_upload_ = 0;
    int64_t n_spmv_ = 0, n_cg_ = 0, n_failed_ = 0, n_uploads_ = 0, n_evict_ = 0,
            n_ticks_ = 0;
    double bytes_done_ = 0.0;
    int64_t t_first_ = 0, t_last_ = 0;
    std::string err_;
    bool dead_ = false;
    int64_t peak_pub_ = 0;   // peak_ as the client side sees it
    std::deque<Done> up_done_;
};

}  // namespace serve
}  // namespace lilac

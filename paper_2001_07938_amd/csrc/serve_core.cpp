// Scheduling core of the request server (see serve_core.h).
#include "serve_core.h"

#include <algorithm>
#include <chrono>

namespace lilac {
namespace serve {

Core::Core(Executor &ex, const Limits &lim) : ex_(ex), lim_(lim)
{
    lim_.max_active = std::max(1, lim_.max_active);
    lim_.pool_capacity = std::max(1, lim_.pool_capacity);
    charged_ = lim_.overhead;
    peak_ = charged_;
    peak_pub_ = peak_;
}

void Core::bump_peak()
{
    if (charged_ <= peak_)
        return;
    peak_ = charged_;
    std::lock_guard<std::mutex> lk(mu_);
    peak_pub_ = peak_;
}

Core::~Core()
{
    for (Request *r : waiting_)
        delete r;
    for (Request *r : incoming_)
        delete r;
    for (auto &act : active_)
        for (Request *r : act)
            delete r;
    for (auto &lane : finishing_)
        for (auto &f : lane)
            for (Request *r : f)
                delete r;
}

int Core::add_matrix(int64_t spmv_bytes, int64_t cg_iter_bytes)
{
    Mat m;
    m.spmv_bytes = spmv_bytes;
    m.cg_iter_bytes = cg_iter_bytes;
    mats_.push_back(m);
    return (int)mats_.size() - 1;
}

// ------------------------------------------------------------ client side

uint64_t Core::submit(Request *r)
{
    std::lock_guard<std::mutex> lk(mu_);
    r->ticket = next_ticket_++;
    if (dead_) {
        status_[r->ticket] = -1;
        n_failed_ += 1;
        delete r;
        return next_ticket_ - 1;
    }
    status_[r->ticket] = 0;
    incoming_.push_back(r);
    work_cv_.notify_one();
    return r->ticket;
}

int Core::poll(uint64_t ticket)
{
    std::lock_guard<std::mutex> lk(mu_);
    auto it = status_.find(ticket);
    return it == status_.end() ? -2 : it->second;
}

int Core::wait(uint64_t ticket)
{
    std::unique_lock<std::mutex> lk(mu_);
    auto it = status_.find(ticket);
    if (it == status_.end())
        return -2;
    done_cv_.wait(lk, [&] { return status_[ticket] != 0; });
    return status_[ticket];
}

void Core::forget(uint64_t ticket)
{
    std::lock_guard<std::mutex> lk(mu_);
    auto it = status_.find(ticket);
    if (it != status_.end() && it->second != 0)
        status_.erase(it);
}

Stats Core::stats()
{
    std::lock_guard<std::mutex> lk(mu_);
    Stats o;
    o.completed = (int64_t)lat_us_.size();
    o.spmv_done = n_spmv_;
    o.cg_done = n_cg_;
    o.failed = n_failed_;
    o.uploads = n_uploads_;
    o.evictions = n_evict_;
    o.ticks = n_ticks_;
    o.planned_peak = peak_pub_;
    o.waited_upload = n_waited_upload_;
    if (!lat_us_.empty()) {
        std::vector<double> v = lat_us_;
        auto pct = [&](double p) {
            const size_t k = std::min(v.size() - 1, (size_t)(p * (double)(v.size() - 1) + 0.5));
            std::nth_element(v.begin(), v.begin() + (std::ptrdiff_t)k, v.end());
            return v[k];
        };
        o.p50_us = pct(0.50);
        o.p99_us = pct(0.99);
        double s = 0.0, mx = 0.0;
        for (double x : lat_us_) {
            s += x;
            mx = std::max(mx, x);
        }
        o.mean_us = s / (double)lat_us_.size();
        o.max_us = mx;
        o.mean_wait_us = wait_sum_us_ / (double)lat_us_.size();
        o.mean_run_us = run_sum_us_ / (double)lat_us_.size();
    }
    const double wall = (double)(t_last_ - t_first_) * 1e-9;
    o.wall_s = wall;
    if (wall > 0) {
        o.req_per_s = (double)o.completed / wall;
        o.solves_per_s = (double)n_cg_ / wall;
        o.gbytes_per_s = bytes_done_ / wall / 1e9;
    }
    return o;
}

void Core::reset_stats()
{
    std::lock_guard<std::mutex> lk(mu_);
    lat_us_.clear();
    wait_sum_us_ = run_sum_us_ = 0.0;
    n_waited_upload_ = 0;
    n_spmv_ = n_cg_ = n_failed_ = n_uploads_ = n_evict_ = n_ticks_ = 0;
    bytes_done_ = 0.0;
    t_first_ = t_last_ = 0;
}

std::string Core::error()
{
    std::lock_guard<std::mutex> lk(mu_);
    return err_;
}

bool Core::dead()
{
    std::lock_guard<std::mutex> lk(mu_);
    return dead_;
}

// ---------------------------------------------------------- executor side

void Core::upload_done(int mid, bool ok, int64_t held_bytes, const std::string &err)
{
    std::lock_guard<std::mutex> lk(mu_);
    up_done_.push_back(Done{mid, ok, held_bytes, err});
    work_cv_.notify_one();
}

// ------------------------------------------------------------- scheduler

int Core::uploading() const
{
    int n = 0;
    for (const Mat &m : mats_)
        n += m.st == UPLOADING;
    return n;
}

bool Core::is_resident(int mid) const { return mats_[(size_t)mid].st != OFF; }
bool Core::is_ready(int mid) const { return mats_[(size_t)mid].st == READY; }

void Core::take_incoming()
{
    std::deque<Request *> in;
    {
        std::lock_guard<std::mutex> lk(mu_);
        in.swap(incoming_);
    }
    int64_t cold = 0;
    for (Request *r : in) {
        Mat &m = mats_[(size_t)r->mid];
        cold += m.st != READY;
        m.queued += 1;
        waiting_.push_back(r);
    }
    if (cold) {
        std::lock_guard<std::mutex> lk(mu_);
        n_waited_upload_ += cold;
    }
}

void Core::collect_uploads()
{
    std::deque<Done> done;
    {
        std::lock_guard<std::mutex> lk(mu_);
        done.swap(up_done_);
    }
    for (const Done &d : done) {
        Mat &m = mats_[(size_t)d.mid];
        if (d.ok) {
            // the upload is over: its reserve becomes what the resident copy
            // really holds (never more than the reserve: the executor
            // enforces it)
            if (d.held > m.charge)
                overruns_ += 1;
            charged_ += d.held - m.charge;
            bump_peak();
            m.charge = d.held;
            m.st = READY;
        } else {
            charged_ -= m.charge;
            m.charge = 0;
            m.st = OFF;
            resident_ -= 1;
            {
                std::lock_guard<std::mutex> lk(mu_);
                err_ = d.err;
            }
            fail_waiting_on(d.mid, d.err);
        }
    }
}

// The idle resident matrix to evict: no admitted or waiting request names
// it; among those, the one whose second most recent use is oldest (LRU-2:
// a matrix used once is evicted before one used twice, which keeps the
// often reused pool resident against one-off uploads), ties by the most
// recent use.  -1 if none.
int Core::pick_victim() const
{
    int best = -1;
    for (int i = 0; i < (int)mats_.size(); ++i) {
        const Mat &m = mats_[(size_t)i];
        if (m.st != READY || m.refs != 0 || m.queued != 0)
            continue;
        if (best < 0)
            best = i;
        else {
            const Mat &b = mats_[(size_t)best];
            if (m.prev_use < b.prev_use ||
                (m.prev_use == b.prev_use && m.last_use < b.last_use))
                best = i;
        }
    }
    return best;
}

void Core::evict(int mid)
{
    Mat &m = mats_[(size_t)mid];
    ex_.evict(mid);
    charged_ -= m.charge;
    m.charge = 0;
    m.st = OFF;
    resident_ -= 1;
    std::lock_guard<std::mutex> lk(mu_);
    n_evict_ += 1;
}

// Frees planned bytes until `need` more fit the budget (and, for an upload,
// until the pool has a free place): idle matrices first, then unused slots.
bool Core::make_room(int64_t need, bool for_upload)
{
    while (charged_ + need > lim_.budget ||
           (for_upload && resident_ >= lim_.pool_capacity)) {
        const int v = pick_victim();
        if (v >= 0) {
            evict(v);
            continue;
        }
        if (for_upload && resident_ >= lim_.pool_capacity)
            return false;
        // unused slots give their memory back
        int freed = -1;
        for (int s : free_slots_)
            if (slots_[(size_t)s].charge > 0) {
                freed = s;
                break;
            }
        if (freed < 0)
            return false;
        ex_.release_slot(freed);
        charged_ -= slots_[(size_t)freed].charge;
        slots_[(size_t)freed].charge = 0;
    }
    return true;
}

void Core::fail_waiting_on(int mid, const std::string &why)
{
    (void)why;
    for (auto it = waiting_.begin(); it != waiting_.end();) {
        if ((*it)->mid == mid) {
            Request *r = *it;
            it = waiting_.erase(it);
            mats_[(size_t)mid].queued -= 1;
            r->failed = true;
            finish(r, ex_.now_ns());
        } else {
            ++it;
        }
    }
}

bool Core::try_upload(int mid)
{
    Mat &m = mats_[(size_t)mid];
    const int64_t reserve = ex_.upload_reserve(mid);
    if (reserve + lim_.overhead > lim_.budget) {
        {
            std::lock_guard<std::mutex> lk(mu_);
            err_ = "matrix " + std::to_string(mid) + " needs " + std::to_string(reserve) +
                   " bytes, more than the server's HBM budget";
        }
        fail_waiting_on(mid, "matrix larger than the budget");
        return false;
    }
    if (!make_room(reserve, true))
        return false;  // again once something is idle
    m.st = UPLOADING;
    m.charge = reserve;
    charged_ += reserve;
    bump_peak();
    resident_ += 1;
    {
        std::lock_guard<std::mutex> lk(mu_);
        n_uploads_ += 1;
    }
    ex_.start_upload(mid);
    return true;
}

bool Core::get_slot(Request *r)
{
    int s;
    if (!free_slots_.empty()) {
        // the free slot that already holds the most memory
        auto best = free_slots_.begin();
        for (auto it = free_slots_.begin(); it != free_slots_.end(); ++it)
            if (slots_[(size_t)*it].charge > slots_[(size_t)*best].charge)
                best = it;
        s = *best;
    } else {
        if ((int)slots_.size() >= lim_.max_active)
            return false;
        slots_.push_back(Slot());
        s = (int)slots_.size() - 1;
        free_slots_.push_back(s);
    }
    // taken off the free list first, so that making room cannot free it
    free_slots_.erase(std::find(free_slots_.begin(), free_slots_.end(), s));
    const int64_t need = ex_.slot_need(s, r->mid);
    const int64_t grow = std::max<int64_t>(0, need - slots_[(size_t)s].charge);
    if (grow > 0) {
        // room for the slot (the request's own matrix is queued, so it is
        // never the one evicted)
        if (!make_room(grow, false)) {
            free_slots_.push_back(s);
            return false;
        }
        ex_.prepare_slot(s, r->mid);
        charged_ += grow;
        bump_peak();
        slots_[(size_t)s].charge += grow;
    }
    slots_[(size_t)s].busy = true;
    r->slot = s;
    return true;
}

void Core::finish(Request *r, int64_t t)
{
    Mat &m = mats_[(size_t)r->mid];
    if (r->slot >= 0) {
        m.refs -= 1;
        slots_[(size_t)r->slot].busy = false;
        free_slots_.push_back(r->slot);
    }
    {
        std::lock_guard<std::mutex> lk(mu_);
        if (r->failed) {
            status_[r->ticket] = -1;
            n_failed_ += 1;
        } else {
            status_[r->ticket] = 1;
            lat_us_.push_back((double)(t - r->t_arr) * 1e-3);
            wait_sum_us_ += (double)(r->t_adm - r->t_arr) * 1e-3;
            run_sum_us_ += (double)(t - r->t_adm) * 1e-3;
            if (r->kind == kCg) {
                n_cg_ += 1;
                bytes_done_ += (double)r->iters * (double)m.cg_iter_bytes;
            } else {
                n_spmv_ += 1;
                bytes_done_ += (double)m.spmv_bytes;
            }
            if (!t_first_ || r->t_arr < t_first_)
                t_first_ = r->t_arr;
            t_last_ = std::max(t_last_, t);
        }
    }
    done_cv_.notify_all();
    delete r;
}

void Core::complete(int lane, int tick)
{
    if (!pending_[lane][tick])
        return;
    ex_.wait_tick(lane, tick);
    const int64_t t = ex_.now_ns();
    for (Request *r : finishing_[lane][tick])
        finish(r, t);
    finishing_[lane][tick].clear();
    pending_[lane][tick] = false;
}

// Launches the lane's next tick if its tick buffer is free (a lane keeps at
// most two ticks on the device, so the next one is queued behind the
// running one).
bool Core::launch(int lane)
{
    std::vector<Request *> &act = active_[lane];
    if (act.empty())
        return false;
    const int tk = tick_no_[lane] & 1;
    if (pending_[lane][tk]) {
        if (!ex_.tick_done(lane, tk))
            return false;
        complete(lane, tk);
    }
    ex_.launch_tick(lane, tk, act);
    pending_[lane][tk] = true;
    {
        std::lock_guard<std::mutex> lk(mu_);
        n_ticks_ += 1;
    }
    // requests whose last step is in this tick leave the active set now;
    // they finish when the tick does
    std::vector<Request *> still;
    for (Request *r : act) {
        if (r->kind == kCg) {
            r->iter += 1;
            if (r->iter < r->iters) {
                still.push_back(r);
                continue;
            }
        }
        finishing_[lane][tk].push_back(r);
    }
    act.swap(still);
    tick_no_[lane] += 1;
    return true;
}

bool Core::busy() const
{
    for (int l = 0; l < kLanes; ++l)
        if (pending_[l][0] || pending_[l][1])
            return true;
    return false;
}

bool Core::step()
{
    take_incoming();
    collect_uploads();
    bool worked = false;
    // ticks that are over give their requests back
    for (int l = 0; l < kLanes; ++l)
        for (int t = 0; t < 2; ++t)
            if (pending_[l][t] && ex_.tick_done(l, t)) {
                complete(l, t);
                worked = true;
            }
    // admission in arrival order; a request whose matrix is not resident
    // does not hold up the ones behind it
    for (auto it = waiting_.begin(); it != waiting_.end();) {
        Request *r = *it;
        Mat &m = mats_[(size_t)r->mid];
        if (m.st == OFF) {
            const size_t before = waiting_.size();
            if (try_upload(r->mid))
                worked = true;
            if (waiting_.size() != before) {
                // the matrix can never fit: its requests failed and left
                // the queue; look at the queue again from its start
                worked = true;
                it = waiting_.begin();
                continue;
            }
            ++it;
            continue;
        }
        if (m.st != READY) {
            ++it;
            continue;
        }
        if (lim_.fifo) {
            if (!get_slot(r))
                break;
            it = waiting_.erase(it);
            m.queued -= 1;
            m.refs += 1;
            m.prev_use = m.last_use;
            m.last_use = ++use_clock_;
            r->t_adm = ex_.now_ns();
            ex_.run_one(r);
            finish(r, ex_.now_ns());
            return true;  // one request per round
        }
        if (active() >= lim_.max_active)
            break;
        if (!get_slot(r))
            break;
        m.refs += 1;
        m.queued -= 1;
        m.prev_use = m.last_use;
        m.last_use = ++use_clock_;
        r->t_adm = ex_.now_ns();
        active_[ex_.lane_of(r->mid)].push_back(r);
        it = waiting_.erase(it);
        worked = true;
    }
    for (int l = 0; l < kLanes; ++l)
        if (launch(l))
            worked = true;
    return worked;
}

void Core::wait_for_work(int64_t max_ns)
{
    // a deadline on the system clock: a new request or upload result wakes
    // the wait at once, the deadline only bounds an idle poll (and this form
    // is the one the thread sanitizer of the toolchain understands)
    std::unique_lock<std::mutex> lk(mu_);
    work_cv_.wait_until(lk, std::chrono::system_clock::now() + std::chrono::nanoseconds(max_ns),
                        [&] { return !incoming_.empty() || !up_done_.empty(); });
}

void Core::wake()
{
    std::lock_guard<std::mutex> lk(mu_);
    work_cv_.notify_all();
}

void Core::shutdown()
{
    take_incoming();
    collect_uploads();
    for (Request *r : waiting_) {
        mats_[(size_t)r->mid].queued -= 1;
        r->failed = true;
        finish(r, ex_.now_ns());
    }
    waiting_.clear();
    for (int l = 0; l < kLanes; ++l) {
        while (!active_[l].empty()) {
            if (!launch(l))
                complete(l, tick_no_[l] & 1);   // wait for the buffer, then launch
        }
        complete(l, 0);
        complete(l, 1);
    }
}

void Core::die(const std::string &msg)
{
    std::lock_guard<std::mutex> lk(mu_);
    err_ = msg;
    dead_ = true;
    for (auto &kv : status_)
        if (kv.second == 0) {
            kv.second = -1;
            n_failed_ += 1;
        }
    done_cv_.notify_all();
}

}  // namespace serve
}  // namespace lilac

// CPU tests of the request server's scheduling core (serve_core.cpp, built
// with g++; no GPU).  A simulated executor models the device: uploads that
// take time and hold a transient reserve before settling to their final
// size, evictions, slot memory, ticks that run one after another, all in
// virtual time, so every schedule is exact and repeatable.  Checked: the
// device model never holds more than the budget, the plan never promises
// more than the budget, nothing in use or queued is evicted, the eviction
// order is LRU-2, slots bound the requests in a tick, every request ends
// exactly once, and a matrix that can never fit fails cleanly.  A last test
// runs the core with real threads (scheduler, two upload threads, several
// clients) for the thread sanitizer.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "serve_core.h"

using namespace lilac::serve;

static int g_fail = 0;
#define CHECK(c)                                                                    \
    do {                                                                            \
        if (!(c)) {                                                                 \
            std::fprintf(stderr, "FAIL %s:%d: %s\n", __FILE__, __LINE__, #c);       \
            ++g_fail;                                                               \
            return;                                                                 \
        }                                                                           \
    } while (0)

// ------------------------------------------------------------ simulation

struct MatModel {
    int64_t reserve = 0;   // bytes set aside before the upload
    int64_t final = 0;     // bytes the resident copy holds
    int64_t up_ns = 0;     // upload time
    int64_t work_ns = 0;   // one product (or one CG iteration) in a tick
    int lane = 0;          // 0 light, 1 heavy
};

class SimExec : public Executor {
  public:
    SimExec(std::vector<MatModel> mats, int64_t budget, int64_t slot_bytes)
        : m(std::move(mats)), budget(budget), slot_bytes(slot_bytes),
          held(m.size(), 0), uploading(m.size(), false)
    {
    }
    Core *core = nullptr;
    std::vector<MatModel> m;
    int64_t budget, slot_bytes;
    int64_t t = 0;                 // virtual clock
    int64_t used = 0, peak = 0;    // modelled device bytes
    std::vector<int64_t> held;
    std::vector<bool> uploading;
    std::vector<int64_t> slot_held;
    std::multimap<int64_t, int> up_events;   // completion time -> matrix
    int64_t gpu_free_at[kLanes] = {0, 0};    // a lane's ticks run one after another
    int64_t tick_end[kLanes][2] = {{0, 0}, {0, 0}};
    std::set<int> tick_mats[kLanes][2];      // matrices a pending tick reads
    std::vector<int> evicted;
    int max_in_tick = 0, ticks = 0, fifo_runs = 0;
    bool violated = false;
    std::string why;

    void charge(int64_t b)
    {
        used += b;
        peak = std::max(peak, used);
        if (used > budget) {
            violated = true;
            why = "device model over budget";
        }
    }
    void bad(const std::string &w)
    {
        violated = true;
        why = w;
    }

    int64_t now_ns() override { return t; }
    int64_t upload_reserve(int mid) override { return m[(size_t)mid].reserve; }
    void start_upload(int mid) override
    {
        if (held[(size_t)mid] || uploading[(size_t)mid])
            bad("upload of a resident matrix");
        uploading[(size_t)mid] = true;
        charge(m[(size_t)mid].reserve);   // the transient peak of the build
        up_events.emplace(t + m[(size_t)mid].up_ns, mid);
    }
    // uploads whose time has come report back (as the upload threads do)
    void deliver(int64_t until)
    {
        while (!up_events.empty() && up_events.begin()->first <= until) {
            const int mid = up_events.begin()->second;
            up_events.erase(up_events.begin());
            const MatModel &mm = m[(size_t)mid];
            used -= mm.reserve - mm.final;
            held[(size_t)mid] = mm.final;
            uploading[(size_t)mid] = false;
            core->upload_done(mid, true, mm.final, "");
        }
    }
    void evict(int mid) override
    {
        if (!held[(size_t)mid])
            bad("eviction of a matrix that is not resident");
        for (int l = 0; l < kLanes; ++l)
            for (int k = 0; k < 2; ++k)
                if (tick_end[l][k] > t && tick_mats[l][k].count(mid))
                    bad("eviction of a matrix a running tick reads");
        used -= held[(size_t)mid];
        held[(size_t)mid] = 0;
        evicted.push_back(mid);
    }
    int64_t slot_need(int, int) override { return slot_bytes; }
    void prepare_slot(int slot, int) override
    {
        if ((int)slot_held.size() <= slot)
            slot_held.resize((size_t)slot + 1, 0);
        charge(slot_bytes - slot_held[(size_t)slot]);
        slot_held[(size_t)slot] = slot_bytes;
    }
    void release_slot(int slot) override
    {
        used -= slot_held[(size_t)slot];
        slot_held[(size_t)slot] = 0;
    }
    int lane_of(int mid) override { return m[(size_t)mid].lane; }
    void launch_tick(int lane, int tick, const std::vector<Request *> &reqs) override
    {
        if (tick_end[lane][tick] > t)
            bad("tick buffer reused while its tick runs");
        int64_t d = 2000;
        tick_mats[lane][tick].clear();
        for (Request *r : reqs) {
            if (!held[(size_t)r->mid])
                bad("tick reads a matrix that is not resident");
            if (r->slot < 0 || r->slot >= (int)slot_held.size() || !slot_held[(size_t)r->slot])
                bad("request without slot memory");
            if (m[(size_t)r->mid].lane != lane)
                bad("request in the wrong lane");
            d += m[(size_t)r->mid].work_ns;
            tick_mats[lane][tick].insert(r->mid);
        }
        gpu_free_at[lane] = std::max(gpu_free_at[lane], t) + d;
        tick_end[lane][tick] = gpu_free_at[lane];
        max_in_tick = std::max(max_in_tick, (int)reqs.size());
        ticks += 1;
    }
    bool tick_done(int lane, int tick) override { return tick_end[lane][tick] <= t; }
    void wait_tick(int lane, int tick) override
    {
        if (tick_end[lane][tick] > t) {
            deliver(tick_end[lane][tick]);
            t = tick_end[lane][tick];
        }
    }
    int64_t next_tick_end() const
    {
        int64_t e = INT64_MAX;
        for (int l = 0; l < kLanes; ++l)
            for (int k = 0; k < 2; ++k)
                if (tick_end[l][k] > t)
                    e = std::min(e, tick_end[l][k]);
        return e;
    }
    void run_one(Request *r) override
    {
        if (!held[(size_t)r->mid])
            bad("plain path on a matrix that is not resident");
        t += 1000 + m[(size_t)r->mid].work_ns * (r->kind == kCg ? r->iters : 1);
        fifo_runs += 1;
    }
};

struct Arrival {
    int64_t t;
    int kind, mid, iters;
};

// Runs the core until every request ended; returns the tickets in order.
static std::vector<uint64_t> simulate(Core &core, SimExec &ex, std::vector<Arrival> arr)
{
    std::stable_sort(arr.begin(), arr.end(),
                     [](const Arrival &a, const Arrival &b) { return a.t < b.t; });
    std::vector<uint64_t> tickets;
    size_t next = 0;
    for (int guard = 0; guard < 10000000; ++guard) {
        while (next < arr.size() && arr[next].t <= ex.t) {
            auto *r = new Request();
            r->kind = arr[next].kind;
            r->mid = arr[next].mid;
            r->iters = arr[next].iters;
            r->t_arr = arr[next].t;
            tickets.push_back(core.submit(r));
            ++next;
        }
        ex.deliver(ex.t);
        if (core.step())
            continue;
        // idle: jump to the next event
        int64_t tn = INT64_MAX;
        if (next < arr.size())
            tn = arr[next].t;
        if (!ex.up_events.empty())
            tn = std::min(tn, ex.up_events.begin()->first);
        tn = std::min(tn, ex.next_tick_end());
        if (tn == INT64_MAX)
            break;
        ex.t = std::max(ex.t, tn);
    }
    return tickets;
}

static Limits limits(int64_t budget, int max_active, int pool, bool fifo = false)
{
    Limits l;
    l.budget = budget;
    l.max_active = max_active;
    l.pool_capacity = pool;
    l.fifo = fifo;
    l.overhead = 1000;
    return l;
}

static void add_all(Core &core, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        core.add_matrix(100, 200);
}

// ------------------------------------------------------------ the tests

// Four matrices, room for two at a time: uploads wait for idle matrices to
// go, the device model never passes the budget, all requests complete.
static void test_budget_exhaustion()
{
    std::vector<MatModel> mm(4, MatModel{600000, 450000, 50000, 3000});
    const int64_t budget = 1000 + 2 * 600000 + 4 * 10000;
    SimExec ex(mm, budget, 10000);
    Core core(ex, limits(budget, 4, 8));
    ex.core = &core;
    add_all(core, 4);
    std::vector<Arrival> a;
    for (int i = 0; i < 40; ++i)
        a.push_back({i * 7000, i % 3 == 0 ? kCg : kSpmv, i % 4, 5});
    auto tk = simulate(core, ex, a);
    CHECK(!ex.violated);
    CHECK(ex.peak <= budget);
    CHECK(core.planned_peak() <= budget);
    for (uint64_t t : tk)
        CHECK(core.poll(t) == 1);
    CHECK(core.stats().completed == 40);
    CHECK(!ex.evicted.empty());
    CHECK(core.reserve_overruns() == 0);
    // what stays resident is charged at its final size, not its reserve
    for (int mid = 0; mid < 4; ++mid)
        if (core.is_ready(mid))
            CHECK(core.matrix_charge(mid) == 450000);
}

// LRU-2: with A used twice and B, C once each, a fourth matrix evicts B
// (oldest among those used once), where plain LRU would evict A.
static void test_lru2_victim()
{
    std::vector<MatModel> mm(4, MatModel{1000, 1000, 1000, 1000});
    SimExec ex(mm, 1 << 30, 100);
    Core core(ex, limits(1 << 30, 8, 3));
    ex.core = &core;
    add_all(core, 4);
    // A, A, B, C well apart (each finishes before the next), then D
    std::vector<Arrival> a = {{0, kSpmv, 0, 1},      {100000, kSpmv, 0, 1},
                              {200000, kSpmv, 1, 1}, {300000, kSpmv, 2, 1},
                              {400000, kSpmv, 3, 1}};
    simulate(core, ex, a);
    CHECK(!ex.violated);
    CHECK(ex.evicted.size() == 1);
    CHECK(ex.evicted[0] == 1);
    CHECK(core.is_resident(0) && core.is_resident(2) && core.is_resident(3));
}

// A matrix with admitted or queued requests is never evicted: with a pool
// of one, a request on B waits until the long CG on A has finished.
static void test_no_eviction_in_use()
{
    std::vector<MatModel> mm(2, MatModel{1000, 1000, 1000, 50000});
    SimExec ex(mm, 1 << 30, 100);
    Core core(ex, limits(1 << 30, 8, 1));
    ex.core = &core;
    add_all(core, 2);
    std::vector<Arrival> a = {{0, kCg, 0, 20}, {5000, kSpmv, 1, 1}, {6000, kSpmv, 0, 1}};
    auto tk = simulate(core, ex, a);
    CHECK(!ex.violated);
    for (uint64_t t : tk)
        CHECK(core.poll(t) == 1);
    CHECK(ex.evicted.size() == 1 && ex.evicted[0] == 0);
    CHECK(core.stats().completed == 3);
}

// Slots: at most max_active requests in any tick; requests are admitted in
// arrival order, so the first ones finish first.
static void test_slot_limit()
{
    std::vector<MatModel> mm(1, MatModel{1000, 1000, 1000, 500});
    SimExec ex(mm, 1 << 30, 100);
    Core core(ex, limits(1 << 30, 2, 4));
    ex.core = &core;
    add_all(core, 1);
    std::vector<Arrival> a;
    for (int i = 0; i < 6; ++i)
        a.push_back({0, kCg, 0, 10});
    auto tk = simulate(core, ex, a);
    CHECK(!ex.violated);
    CHECK(ex.max_in_tick == 2);
    for (uint64_t t : tk)
        CHECK(core.poll(t) == 1);
    // 6 solves of 10 iterations, two at a time: at least 30 ticks
    CHECK(ex.ticks >= 30);
}

// A matrix whose reserve exceeds the budget fails its requests; the others
// still complete and nothing is charged for it.
static void test_too_large_fails()
{
    std::vector<MatModel> mm = {MatModel{5000, 4000, 100, 100},
                                MatModel{1 << 20, 1 << 20, 100, 100}};
    const int64_t budget = 100000;
    SimExec ex(mm, budget, 100);
    Core core(ex, limits(budget, 4, 4));
    ex.core = &core;
    add_all(core, 2);
    std::vector<Arrival> a = {{0, kSpmv, 1, 1}, {0, kSpmv, 0, 1}, {10, kSpmv, 1, 1}};
    auto tk = simulate(core, ex, a);
    CHECK(!ex.violated);
    CHECK(core.poll(tk[0]) == -1);
    CHECK(core.poll(tk[1]) == 1);
    CHECK(core.poll(tk[2]) == -1);
    CHECK(core.stats().failed == 2);
    CHECK(!core.is_resident(1));
    CHECK(core.planned_bytes() <= budget);
}

// Slots give their memory back to an upload when no matrix can go.
static void test_slots_released_for_uploads()
{
    std::vector<MatModel> mm(2, MatModel{50000, 40000, 1000, 1000});
    const int64_t budget = 1000 + 50000 + 40000 + 3 * 8000;
    SimExec ex(mm, budget, 8000);
    Core core(ex, limits(budget, 8, 4));
    ex.core = &core;
    add_all(core, 2);
    std::vector<Arrival> a;
    for (int i = 0; i < 8; ++i)   // many slots on matrix 0 at once
        a.push_back({0, kSpmv, 0, 1});
    a.push_back({200000, kSpmv, 1, 1});
    auto tk = simulate(core, ex, a);
    CHECK(!ex.violated);
    for (uint64_t t : tk)
        CHECK(core.poll(t) == 1);
    CHECK(ex.peak <= budget);
}

// The plain path runs one request at a time and launches no tick.
static void test_fifo()
{
    std::vector<MatModel> mm(3, MatModel{1000, 1000, 1000, 1000});
    SimExec ex(mm, 1 << 30, 100);
    Core core(ex, limits(1 << 30, 8, 2, true));
    ex.core = &core;
    add_all(core, 3);
    std::vector<Arrival> a;
    for (int i = 0; i < 12; ++i)
        a.push_back({i * 100, i % 2 ? kCg : kSpmv, i % 3, 4});
    auto tk = simulate(core, ex, a);
    CHECK(!ex.violated);
    CHECK(ex.ticks == 0 && ex.fifo_runs == 12);
    for (uint64_t t : tk)
        CHECK(core.poll(t) == 1);
}

// Random Poisson traces over many matrices under a tight budget and pool:
// the invariants hold and every request completes.
static void test_random_traces()
{
    for (int seed = 1; seed <= 12; ++seed) {
        std::mt19937_64 rng((uint64_t)seed);
        const int nm = 30;
        std::vector<MatModel> mm;
        for (int i = 0; i < nm; ++i) {
            const int64_t fin = 20000 + (int64_t)(rng() % 200000);
            mm.push_back(MatModel{fin + fin / 4, fin, 1000 + fin / 10,
                                  200 + (int64_t)(rng() % 5000), (int)(rng() % 2)});
        }
        const int64_t budget = 1000 + 900000 + (int64_t)(rng() % 400000);
        SimExec ex(mm, budget, 3000);
        Core core(ex, limits(budget, 1 + (int)(rng() % 16), 2 + (int)(rng() % 8)));
        ex.core = &core;
        add_all(core, (size_t)nm);
        std::vector<Arrival> a;
        int64_t t = 0;
        std::exponential_distribution<double> gap(1.0 / 3000.0);
        for (int i = 0; i < 600; ++i) {
            t += (int64_t)gap(rng);
            const int mid = (rng() % 10 < 9) ? (int)(rng() % 8) : 8 + (int)(rng() % (nm - 8));
            a.push_back({t, rng() % 5 == 0 ? kCg : kSpmv, mid, 1 + (int)(rng() % 20)});
        }
        auto tk = simulate(core, ex, a);
        if (ex.violated)
            std::fprintf(stderr, "seed %d: %s\n", seed, ex.why.c_str());
        CHECK(!ex.violated);
        CHECK(ex.peak <= budget);
        CHECK(core.planned_peak() <= budget);
        CHECK(core.reserve_overruns() == 0);
        int done = 0;
        for (uint64_t x : tk)
            done += core.poll(x) == 1;
        CHECK(done == 600);
        CHECK(core.active() == 0 && core.waiting() == 0);
    }
}

// ------------------------------------------------------ real threads

// The executor the threaded test uses: uploads on two threads of its own,
// ticks and evictions as short sleeps; device bytes counted atomically.
class ThreadExec : public Executor {
  public:
    explicit ThreadExec(int n) : held(n) {}
    Core *core = nullptr;
    std::vector<std::atomic<int64_t>> held;
    std::atomic<int64_t> used{0}, peak{0};
    int64_t budget = 0;
    std::mutex mu;
    std::condition_variable cv;
    std::vector<int> q;
    bool stop = false;
    std::thread up[2];

    void start()
    {
        for (auto &u : up)
            u = std::thread([this] {
                while (true) {
                    int mid;
                    {
                        std::unique_lock<std::mutex> lk(mu);
                        cv.wait(lk, [&] { return stop || !q.empty(); });
                        if (stop)
                            return;
                        mid = q.back();
                        q.pop_back();
                    }
                    std::this_thread::sleep_for(std::chrono::microseconds(50));
                    held[(size_t)mid] = 900;
                    used -= 100;
                    core->upload_done(mid, true, 900, "");
                }
            });
    }
    void finish()
    {
        {
            std::lock_guard<std::mutex> lk(mu);
            stop = true;
        }
        cv.notify_all();
        for (auto &u : up)
            u.join();
    }
    void add(int64_t b)
    {
        const int64_t u = (used += b);
        int64_t p = peak.load();
        while (u > p && !peak.compare_exchange_weak(p, u)) {
        }
    }
    int64_t now_ns() override
    {
        return std::chrono::duration_cast<std::chrono::nanoseconds>(
                   std::chrono::steady_clock::now().time_since_epoch())
            .count();
    }
    int64_t upload_reserve(int) override { return 1000; }
    void start_upload(int mid) override
    {
        add(1000);
        std::lock_guard<std::mutex> lk(mu);
        q.push_back(mid);
        cv.notify_one();
    }
    void evict(int mid) override
    {
        used -= held[(size_t)mid];
        held[(size_t)mid] = 0;
    }
    int64_t slot_need(int, int) override { return 100; }
    void prepare_slot(int, int) override { add(100); }
    void release_slot(int) override { used -= 100; }
    int lane_of(int mid) override { return mid % 2; }
    void launch_tick(int, int, const std::vector<Request *> &) override {}
    bool tick_done(int, int) override { return true; }
    void wait_tick(int, int) override { std::this_thread::sleep_for(std::chrono::microseconds(20)); }
    void run_one(Request *) override {}
};

static void test_threads()
{
    const int nm = 12;
    ThreadExec ex(nm);
    const int64_t budget = 1000 + 4 * 1000 + 8 * 100;
    ex.budget = budget;
    Core core(ex, limits(budget, 8, 4));
    ex.core = &core;
    add_all(core, nm);
    ex.start();
    std::atomic<bool> stop{false};
    std::thread sched([&] {
        while (!stop.load())
            if (!core.step())
                core.wait_for_work(core.busy() ? 20000 : 100000);
        core.shutdown();
    });
    std::vector<std::thread> clients;
    std::atomic<int> ok{0};
    for (int c = 0; c < 4; ++c)
        clients.emplace_back([&, c] {
            std::mt19937 rng((unsigned)c);
            for (int i = 0; i < 150; ++i) {
                auto *r = new Request();
                r->kind = (rng() % 4 == 0) ? kCg : kSpmv;
                r->mid = (int)(rng() % nm);
                r->iters = 3;
                r->t_arr = ex.now_ns();
                const uint64_t t = core.submit(r);
                if (core.wait(t) == 1)
                    ok += 1;
                core.forget(t);
                (void)core.stats();
            }
        });
    for (auto &c : clients)
        c.join();
    stop.store(true);
    core.wake();
    sched.join();
    ex.finish();
    CHECK(ok.load() == 600);
    CHECK(ex.peak.load() <= budget);
}

// Two lanes: short requests do not wait out the long ticks of a heavy
// solve; they finish while it still runs, and the heavy lane's ticks are
// never slowed by them.
static void test_lanes_keep_short_requests_short()
{
    std::vector<MatModel> mm = {MatModel{1000, 1000, 1000, 100000, 1},
                                MatModel{1000, 1000, 1000, 1000, 0},
                                MatModel{1000, 1000, 1000, 1000, 0}};
    SimExec ex(mm, 1 << 30, 100);
    Core core(ex, limits(1 << 30, 16, 4));
    ex.core = &core;
    add_all(core, 3);
    std::vector<Arrival> a = {{0, kCg, 0, 30}};
    for (int i = 0; i < 20; ++i)
        a.push_back({200000 + i * 50000, i % 3 == 0 ? kCg : kSpmv, 1 + i % 2, 5});
    auto tk = simulate(core, ex, a);
    CHECK(!ex.violated);
    for (uint64_t t : tk)
        CHECK(core.poll(t) == 1);
    const Stats st = core.stats();
    // the heavy solve alone: 30 ticks of ~102 us; each short request a few
    // light ticks of ~3 us.  Without lanes a short one would take at least
    // one heavy tick per step.
    CHECK(st.max_us >= 30 * 100.0);
    CHECK(st.p50_us < 100.0);
}

int main()
{
    test_budget_exhaustion();
    test_lru2_victim();
    test_no_eviction_in_use();
    test_slot_limit();
    test_too_large_fails();
    test_slots_released_for_uploads();
    test_fifo();
    test_lanes_keep_short_requests_short();
    test_random_traces();
    test_threads();
    if (g_fail) {
        std::fprintf(stderr, "%d check(s) failed\n", g_fail);
        return 1;
    }
    std::printf("serve core ok\n");
    return 0;
}

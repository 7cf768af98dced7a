// Page-protection write tracking (see marshal.h).
#include "marshal.h"

#include <atomic>
#include <csignal>
#include <cstring>
#include <sys/mman.h>
#include <unistd.h>

namespace lilac {
namespace {

constexpr int kMaxRanges = 4096;

struct Range {
    std::atomic<const void *> owner{nullptr};
    int kind = 0;
    uintptr_t page_lo = 0, page_hi = 0;  // page-aligned cover of the range
    std::atomic<int> armed{0};
    std::atomic<int> dirty{0};
};

Range g_ranges[kMaxRanges];
std::atomic<int> g_nranges{0};
std::atomic<uint64_t> g_faults{0};
struct sigaction g_prev;
bool g_installed = false;

uintptr_t page_size()
{
    static uintptr_t ps = (uintptr_t)sysconf(_SC_PAGESIZE);
    return ps;
}

void set_prot(const Range &r, int prot)
{
    (void)mprotect((void *)r.page_lo, r.page_hi - r.page_lo, prot);
}

// SIGSEGV handler: a write to an armed page marks every armed range that
// covers the page dirty and makes it writable; the write then retries.  A
// fault outside every armed range goes to the previous handler.
void on_fault(int sig, siginfo_t *info, void *uctx)
{
    const uintptr_t a = (uintptr_t)info->si_addr;
    bool hit = false;
    const int n = g_nranges.load(std::memory_order_acquire);
    for (int i = 0; i < n; ++i) {
        Range &r = g_ranges[i];
        if (!r.owner.load(std::memory_order_acquire) ||
            !r.armed.load(std::memory_order_acquire))
            continue;
        if (a >= r.page_lo && a < r.page_hi) {
            r.dirty.store(1, std::memory_order_release);
            r.armed.store(0, std::memory_order_release);
            set_prot(r, PROT_READ | PROT_WRITE);
            hit = true;
        }
    }
    if (hit) {
        g_faults.fetch_add(1, std::memory_order_relaxed);
        return;
    }
    // not ours: hand over to whoever was there before
    if (g_prev.sa_flags & SA_SIGINFO) {
        if (g_prev.sa_sigaction) {
            g_prev.sa_sigaction(sig, info, uctx);
            return;
        }
    } else if (g_prev.sa_handler != SIG_DFL && g_prev.sa_handler != SIG_IGN) {
        g_prev.sa_handler(sig);
        return;
    }
    signal(sig, SIG_DFL);
    raise(sig);
}

void install()
{
    if (g_installed)
        return;
    struct sigaction sa;
    std::memset(&sa, 0, sizeof(sa));
    sa.sa_sigaction = on_fault;
    sa.sa_flags = SA_SIGINFO | SA_NODEFER;
    sigemptyset(&sa.sa_mask);
    sigaction(SIGSEGV, &sa, &g_prev);
    g_installed = true;
}

// Two ranges whose page covers overlap must be armed and disarmed together,
// otherwise re-arming one would silently re-protect a page the other still
// needs writable.  Arming below re-protects only this owner's ranges; a
// shared page written once marks both owners dirty, which is conservative.

}  // namespace

bool marshal_track_range(const void *owner, int kind, const void *p,
                         size_t bytes)
{
    if (!owner || !p || bytes == 0)
        return false;
    install();
    const uintptr_t ps = page_size();
    const uintptr_t lo = (uintptr_t)p & ~(ps - 1);
    const uintptr_t hi = ((uintptr_t)p + bytes + ps - 1) & ~(ps - 1);
    int slot = -1;
    const int n = g_nranges.load(std::memory_order_acquire);
    for (int i = 0; i < n; ++i)
        if (!g_ranges[i].owner.load(std::memory_order_acquire)) {
            slot = i;
            break;
        }
    if (slot < 0) {
        if (n >= kMaxRanges)
            return false;
        slot = n;
    }
    Range &r = g_ranges[slot];
    r.kind = kind;
    r.page_lo = lo;
    r.page_hi = hi;
    r.dirty.store(0, std::memory_order_relaxed);
    r.armed.store(0, std::memory_order_relaxed);
    r.owner.store(owner, std::memory_order_release);
    if (slot == n)
        g_nranges.store(n + 1, std::memory_order_release);
    r.armed.store(1, std::memory_order_release);
    set_prot(r, PROT_READ);
    return true;
}

int marshal_take_dirty(const void *owner)
{
    int kinds = 0;
    const int n = g_nranges.load(std::memory_order_acquire);
    for (int i = 0; i < n; ++i) {
        Range &r = g_ranges[i];
        if (r.owner.load(std::memory_order_acquire) == owner &&
            r.dirty.exchange(0, std::memory_order_acq_rel))
            kinds |= r.kind;
    }
    return kinds;
}

void marshal_arm(const void *owner)
{
    const int n = g_nranges.load(std::memory_order_acquire);
    for (int i = 0; i < n; ++i) {
        Range &r = g_ranges[i];
        if (r.owner.load(std::memory_order_acquire) == owner) {
            r.dirty.store(0, std::memory_order_release);
            r.armed.store(1, std::memory_order_release);
            set_prot(r, PROT_READ);
        }
    }
}

void marshal_forget(const void *owner)
{
    const int n = g_nranges.load(std::memory_order_acquire);
    for (int i = 0; i < n; ++i) {
        Range &r = g_ranges[i];
        if (r.owner.load(std::memory_order_acquire) == owner) {
            if (r.armed.exchange(0, std::memory_order_acq_rel))
                set_prot(r, PROT_READ | PROT_WRITE);
            r.owner.store(nullptr, std::memory_order_release);
        }
    }
}

void marshal_reset()
{
    const int n = g_nranges.load(std::memory_order_acquire);
    for (int i = 0; i < n; ++i) {
        Range &r = g_ranges[i];
        if (r.owner.load(std::memory_order_acquire)) {
            if (r.armed.exchange(0, std::memory_order_acq_rel))
                set_prot(r, PROT_READ | PROT_WRITE);
            r.owner.store(nullptr, std::memory_order_release);
        }
    }
}

uint64_t marshal_fault_count() { return g_faults.load(); }

}  // namespace lilac

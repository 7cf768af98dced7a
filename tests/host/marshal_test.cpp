// CPU test of the page-protection write tracker (built with g++ together
// with the library's marshal.cpp; no GPU involved).
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <sys/mman.h>
#include <unistd.h>

#include "marshal.h"

using namespace lilac;

#define CHECK(c)                                                            \
    do {                                                                    \
        if (!(c)) {                                                         \
            std::fprintf(stderr, "FAIL %s:%d: %s\n", __FILE__, __LINE__, #c); \
            return 1;                                                       \
        }                                                                   \
    } while (0)

int main()
{
    const long ps = sysconf(_SC_PAGESIZE);
    // three arrays on separate pages
    char *mem = (char *)mmap(nullptr, 8 * ps, PROT_READ | PROT_WRITE,
                             MAP_PRIVATE | MAP_ANONYMOUS, -1, 0);
    CHECK(mem != MAP_FAILED);
    int *rp = (int *)mem;
    int *col = (int *)(mem + 2 * ps);
    double *vals = (double *)(mem + 4 * ps);
    for (int i = 0; i < 100; ++i) {
        rp[i] = i;
        col[i] = i;
        vals[i] = i;
    }
    int owner_a = 0, owner_b = 0;
    CHECK(marshal_track_range(&owner_a, MARSHAL_STRUCT, rp, 100 * sizeof(int)));
    CHECK(marshal_track_range(&owner_a, MARSHAL_STRUCT, col, 100 * sizeof(int)));
    CHECK(marshal_track_range(&owner_a, MARSHAL_VALS, vals, 100 * sizeof(double)));
    CHECK(!marshal_track_range(&owner_b, MARSHAL_VALS, vals, 0));  // empty range
    // reads do not fault and mark nothing
    long sum = 0;
    for (int i = 0; i < 100; ++i)
        sum += rp[i] + col[i] + (long)vals[i];
    CHECK(sum == 3 * 4950);
    CHECK(marshal_take_dirty(&owner_a) == 0);
    CHECK(marshal_fault_count() == 0);
    // a value write is seen once, as a value change
    vals[7] = 70.0;
    CHECK(vals[7] == 70.0);
    CHECK(marshal_fault_count() == 1);
    vals[8] = 80.0;  // page now writable: no second fault
    CHECK(marshal_fault_count() == 1);
    CHECK(marshal_take_dirty(&owner_a) == MARSHAL_VALS);
    CHECK(marshal_take_dirty(&owner_a) == 0);  // record cleared
    // re-arm (after an upload) and write the structure
    marshal_arm(&owner_a);
    col[3] = 4;
    CHECK(marshal_take_dirty(&owner_a) == MARSHAL_STRUCT);
    marshal_arm(&owner_a);
    rp[99] = 100;
    vals[0] = 1.0;
    CHECK(marshal_take_dirty(&owner_a) == (MARSHAL_STRUCT | MARSHAL_VALS));
    CHECK(marshal_fault_count() == 4);
    // forgetting makes the pages writable without faults
    marshal_arm(&owner_a);
    marshal_forget(&owner_a);
    const unsigned long before = marshal_fault_count();
    col[5] = 9;
    vals[5] = 9.0;
    CHECK(marshal_fault_count() == before);
    CHECK(marshal_take_dirty(&owner_a) == 0);
    // two owners sharing a page: one write marks both (conservative)
    CHECK(marshal_track_range(&owner_a, MARSHAL_VALS, vals, 8));
    CHECK(marshal_track_range(&owner_b, MARSHAL_VALS, vals + 16, 8));
    vals[1] = 2.0;
    CHECK(marshal_take_dirty(&owner_a) == MARSHAL_VALS);
    CHECK(marshal_take_dirty(&owner_b) == MARSHAL_VALS);
    marshal_reset();
    vals[2] = 3.0;
    CHECK(marshal_take_dirty(&owner_a) == 0 && marshal_take_dirty(&owner_b) == 0);
    std::printf("marshal ok\n");
    return 0;
}

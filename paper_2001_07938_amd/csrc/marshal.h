// Host-side write tracking for cached host arrays with page protection, the
// mechanism behind the paper's ReadObject marshaling (section
// "Implementation", LiLAC-How, and section "Data Marshaling"): after a host
// array has been copied to the device its pages are made read-only; the
// first later write faults, the handler records that the array changed and
// makes the pages writable again, and the next library call re-uploads it.
//
// Plain C++ and POSIX, no HIP: the same source is built into the library and
// into a CPU-only test program.
#pragma once

#include <cstddef>
#include <cstdint>

namespace lilac {

// Kinds of tracked range: a change to a structure array (row_ptr, col_idx)
// forces a full re-analysis, a change to the values only a value upload.
enum : int { MARSHAL_STRUCT = 1, MARSHAL_VALS = 2 };

// Register a host range [p, p+bytes) owned by `owner` and arm it (pages made
// read-only).  Returns false when the table is full or the range is empty
// (the range is then simply not tracked).
bool marshal_track_range(const void *owner, int kind, const void *p,
                         size_t bytes);
// Bitwise OR of the kinds of `owner`'s ranges written since they were last
// armed; clears the record.
int marshal_take_dirty(const void *owner);
// Re-arm every range of `owner` (after its data has been re-uploaded).
void marshal_arm(const void *owner);
// Stop tracking `owner` (pages become writable again).
void marshal_forget(const void *owner);
// Make every tracked page writable and forget everything.
void marshal_reset();
// Number of write faults the handler has absorbed (for tests and stats).
uint64_t marshal_fault_count();

}  // namespace lilac

// Host entry points of the device-wide primitives (scan, radix sort) used by
// the RCM pass.  All work is enqueued on `stream`; scratch comes from the
// caller's Scratch object (grow-only device buffer).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rbfs {

// Grow-only device scratch; `get` returns a pointer valid until the next get
// with a larger size.  Memory is freed by release().
struct Scratch {
  void* ptr = nullptr;
  size_t bytes = 0;
  hipError_t get(size_t need, void** out);
  void release();
};

// out[i] = sum of in[0..i) for i in [0, n]; out has n + 1 entries (out[n] is
// the total).  In-place (in == out) is not allowed.
hipError_t scan_exclusive_i32(const int32_t* in, int64_t* out, int64_t n, Scratch& s,
                              hipStream_t stream);
hipError_t scan_exclusive_i64(const int64_t* in, int64_t* out, int64_t n, Scratch& s,
                              hipStream_t stream);

// Stable LSD radix sort of n 64-bit keys on bits [begin_bit, end_bit).  The
// sorted keys end in *keys or *alt; on return *keys points at the sorted
// array and *alt at the other buffer (the two pointers may be swapped).
hipError_t radix_sort_u64(uint64_t** keys, uint64_t** alt, int64_t n, int begin_bit,
                          int end_bit, Scratch& s, hipStream_t stream);

}  // namespace rbfs

// ct_segcopy.h -- internal: copy a few byte ranges with one kernel launch.  Used by the request
// server to move requests' keys and values from device-mapped pinned host memory into a batch's
// staging buffer and the results back, instead of one DMA copy per array.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ct_serve {

struct Seg {
  const void* src;  // device-accessible addresses (device memory or mapped pinned host memory)
  void* dst;
  int64_t bytes;
};

constexpr int kMaxSegs = 16;

// Enqueue one kernel on `s` copying segs[0..n), 0 < n <= kMaxSegs; the ranges must not overlap.
hipError_t segcopy(const Seg* segs, int n, hipStream_t s);

}  // namespace ct_serve

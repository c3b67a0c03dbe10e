// Multi-range copy kernel for the request server (interface in ct_segcopy.h).  Segment y of the
// launch is copied by the blocks with blockIdx.y == y, in the widest unit (16, 8, 4 or 1 bytes)
// that its source, destination and length allow, so a wave reads mapped host memory in 512-byte
// or 1 KiB pieces when the arrays are aligned.
#include "ct_segcopy.h"

namespace ct_serve {

namespace {

constexpr int kCopyBlock = 256;

struct SegList {
  Seg s[kMaxSegs];
};

__global__ __launch_bounds__(kCopyBlock) void k_segcopy(SegList L) {
  const Seg g = L.s[blockIdx.y];
  const uintptr_t a = reinterpret_cast<uintptr_t>(g.src) | reinterpret_cast<uintptr_t>(g.dst) |
                      (uintptr_t)g.bytes;
  const int64_t stride = (int64_t)gridDim.x * kCopyBlock;
  const int64_t first = (int64_t)blockIdx.x * kCopyBlock + threadIdx.x;
  if ((a & 15) == 0) {
    const uint4* s = static_cast<const uint4*>(g.src);
    uint4* d = static_cast<uint4*>(g.dst);
    for (int64_t i = first; i < g.bytes / 16; i += stride) d[i] = s[i];
  } else if ((a & 7) == 0) {
    const uint64_t* s = static_cast<const uint64_t*>(g.src);
    uint64_t* d = static_cast<uint64_t*>(g.dst);
    for (int64_t i = first; i < g.bytes / 8; i += stride) d[i] = s[i];
  } else if ((a & 3) == 0) {
    const uint32_t* s = static_cast<const uint32_t*>(g.src);
    uint32_t* d = static_cast<uint32_t*>(g.dst);
    for (int64_t i = first; i < g.bytes / 4; i += stride) d[i] = s[i];
  } else {
    const uint8_t* s = static_cast<const uint8_t*>(g.src);
    uint8_t* d = static_cast<uint8_t*>(g.dst);
    for (int64_t i = first; i < g.bytes; i += stride) d[i] = s[i];
  }
}

}  // namespace

hipError_t segcopy(const Seg* segs, int n, hipStream_t s) {
  if (n <= 0 || n > kMaxSegs) return hipErrorInvalidValue;
  SegList L{};
  int64_t most = 0;
  for (int i = 0; i < n; ++i) {
    L.s[i] = segs[i];
    if (segs[i].bytes > most) most = segs[i].bytes;
  }
  // enough threads for the largest segment in 8-byte units, at most 512 blocks per segment
  int64_t gx = (most / 8 + kCopyBlock - 1) / kCopyBlock;
  if (gx < 1) gx = 1;
  if (gx > 512) gx = 512;
  k_segcopy<<<dim3((unsigned)gx, (unsigned)n), kCopyBlock, 0, s>>>(L);
  return hipGetLastError();
}

}  // namespace ct_serve

// Host-only stand-in for the few HIP runtime calls the request server makes, so that its
// scheduling logic can be built with g++ and run (also under ThreadSanitizer) without a GPU.
// Copies run at once on the calling thread; an event reports "not ready" for a pseudo-random
// number of queries after it is recorded, so completions arrive late and out of order.
#pragma once
#include <atomic>
#include <cstdint>
#include <cstring>

typedef enum hipError_t { hipSuccess = 0, hipErrorNotReady = 600, hipErrorInvalidValue = 1 } hipError_t;
typedef enum hipMemcpyKind { hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2 } hipMemcpyKind;

struct MockStream { int id; };
struct MockEvent { std::atomic<int> pending{0}; uint32_t seed = 1; };
typedef MockStream* hipStream_t;
typedef MockEvent* hipEvent_t;

#define hipStreamNonBlocking 0x01
#define hipEventDisableTiming 0x02

inline std::atomic<int64_t>& mock_live_streams() { static std::atomic<int64_t> n{0}; return n; }
inline std::atomic<int64_t>& mock_live_events() { static std::atomic<int64_t> n{0}; return n; }

inline hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
inline hipError_t hipSetDevice(int) { return hipSuccess; }
inline hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
  static std::atomic<int> next{0};
  *s = new MockStream{next++};
  ++mock_live_streams();
  return hipSuccess;
}
inline hipError_t hipStreamDestroy(hipStream_t s) { delete s; --mock_live_streams(); return hipSuccess; }
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) {
  *e = new MockEvent();
  ++mock_live_events();
  return hipSuccess;
}
inline hipError_t hipEventDestroy(hipEvent_t e) { delete e; --mock_live_events(); return hipSuccess; }
inline hipError_t hipEventRecord(hipEvent_t e, hipStream_t) {
  e->seed = e->seed * 1103515245u + 12345u;
  e->pending.store((int)((e->seed >> 16) % 7));
  return hipSuccess;
}
inline hipError_t hipEventQuery(hipEvent_t e) {
  int p = e->pending.load();
  if (p > 0) {
    e->pending.store(p - 1);
    return hipErrorNotReady;
  }
  return hipSuccess;
}
// Mapped-memory lookup: every other 16-byte granule counts as pinned, so batches take both the
// copy-kernel path and the DMA path.
inline hipError_t hipHostGetDevicePointer(void** d, void* h, unsigned) {
  if ((reinterpret_cast<uintptr_t>(h) >> 4) & 1) return hipErrorInvalidValue;
  *d = h;
  return hipSuccess;
}
inline hipError_t hipGetLastError() { return hipSuccess; }

inline hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind,
                                 hipStream_t) {
  std::memcpy(dst, src, bytes);
  return hipSuccess;
}

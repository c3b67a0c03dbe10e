// ct_roofline.hip -- measured ceilings for the container kernels (see include/ct_roofline.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "ct.h"
#include "ct_device.h"
#include "ct_roofline.h"

using namespace ct;

namespace {

constexpr int kB = 256;

// G lanes read one line of 16*G bytes; XOR of the line goes to out[i].
template <int G, bool CAS>
__global__ __launch_bounds__(kB) void k_gather(uint4* __restrict__ lines, uint64_t nlines,
                                               const uint64_t* __restrict__ keys, int64_t n,
                                               uint64_t* __restrict__ out) {
  const int sub = threadIdx.x % G;
  const int64_t ng = (int64_t)gridDim.x * (kB / G);
  for (int64_t i = (int64_t)blockIdx.x * (kB / G) + threadIdx.x / G; i < n; i += ng) {
    const uint64_t key = keys[i];
    const uint64_t line = __umul64hi(fmix64(key), nlines);
    const uint4 w = lines[line * G + sub];
    uint64_t x = ((uint64_t)w.y << 32 | w.x) ^ ((uint64_t)w.w << 32 | w.z);
    for (int off = 1; off < G; off <<= 1) x ^= __shfl_xor(x, off, 64);
    if (sub == 0) {
      if (CAS) {
        uint64_t* word = reinterpret_cast<uint64_t*>(&lines[line * G]);
        uint64_t expected = (uint64_t)w.y << 32 | w.x;
        cas64(word, expected, expected ^ key);
        x ^= expected;
      }
      out[i] = x;
    }
  }
}

__global__ __launch_bounds__(kB) void k_cas(uint64_t* __restrict__ words, uint64_t nwords,
                                            const uint64_t* __restrict__ keys, int64_t n) {
  const int64_t nt = (int64_t)gridDim.x * kB;
  for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < n; i += nt) {
    const uint64_t key = keys[i];
    uint64_t* w = words + __umul64hi(fmix64(key), nwords);
    uint64_t expected = 0;
    cas64(w, expected, key);
  }
}

// Fire-and-forget 64-bit atomic min (no returned value) on a random word per key.
__global__ __launch_bounds__(kB) void k_amin(uint64_t* __restrict__ words, uint64_t nwords,
                                             const uint64_t* __restrict__ keys, int64_t n) {
  const int64_t nt = (int64_t)gridDim.x * kB;
  for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < n; i += nt) {
    const uint64_t key = keys[i];
    __hip_atomic_fetch_min(words + __umul64hi(fmix64(key), nwords), key, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
  }
}

__global__ __launch_bounds__(kB) void k_copy(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                             int64_t n16) {
  const int64_t nt = (int64_t)gridDim.x * kB;
  for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < n16; i += nt) dst[i] = src[i];
}

int blocks_for(int64_t items, int per_block, int cap) {
  const int64_t b = (items + per_block - 1) / per_block;
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, cap));
}

ct_status done() { return hipGetLastError() == hipSuccess ? CT_OK : CT_E_HIP; }

template <bool CAS>
ct_status gather(void* lines, int64_t nlines, int32_t line_bytes, const uint64_t* keys, int64_t n,
                 uint64_t* out, void* stream) {
  if (!lines || nlines <= 0 || n < 0 || (n > 0 && (!keys || !out))) return CT_E_INVALID;
  if (line_bytes != 64 && line_bytes != 128) return CT_E_INVALID;
  if (reinterpret_cast<uintptr_t>(lines) % 128) return CT_E_INVALID;
  if (n == 0) return CT_OK;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  uint4* L = static_cast<uint4*>(lines);
  if (line_bytes == 128)
    k_gather<8, CAS><<<blocks_for(n, kB / 8, 16384), kB, 0, s>>>(L, (uint64_t)nlines, keys, n, out);
  else
    k_gather<4, CAS><<<blocks_for(n, kB / 4, 16384), kB, 0, s>>>(L, (uint64_t)nlines, keys, n, out);
  return done();
}

}  // namespace

extern "C" {

ct_status ctr_gather(const void* lines, int64_t nlines, int32_t line_bytes, const uint64_t* keys,
                     int64_t n, uint64_t* out, void* stream) {
  return gather<false>(const_cast<void*>(lines), nlines, line_bytes, keys, n, out, stream);
}

ct_status ctr_gather_cas(void* lines, int64_t nlines, int32_t line_bytes, const uint64_t* keys,
                         int64_t n, uint64_t* out, void* stream) {
  return gather<true>(lines, nlines, line_bytes, keys, n, out, stream);
}

ct_status ctr_cas(void* words, int64_t nwords, const uint64_t* keys, int64_t n, void* stream) {
  if (!words || nwords <= 0 || n < 0 || (n > 0 && !keys)) return CT_E_INVALID;
  if (reinterpret_cast<uintptr_t>(words) % 8) return CT_E_INVALID;
  if (n == 0) return CT_OK;
  k_cas<<<blocks_for(n, kB, 16384), kB, 0, reinterpret_cast<hipStream_t>(stream)>>>(
      static_cast<uint64_t*>(words), (uint64_t)nwords, keys, n);
  return done();
}

ct_status ctr_amin(void* words, int64_t nwords, const uint64_t* keys, int64_t n, void* stream) {
  if (!words || nwords <= 0 || n < 0 || (n > 0 && !keys)) return CT_E_INVALID;
  if (reinterpret_cast<uintptr_t>(words) % 8) return CT_E_INVALID;
  if (n == 0) return CT_OK;
  k_amin<<<blocks_for(n, kB, 16384), kB, 0, reinterpret_cast<hipStream_t>(stream)>>>(
      static_cast<uint64_t*>(words), (uint64_t)nwords, keys, n);
  return done();
}

ct_status ctr_copy(const void* src, void* dst, int64_t bytes, void* stream) {
  if (!src || !dst || bytes < 0 || bytes % 16) return CT_E_INVALID;
  if (reinterpret_cast<uintptr_t>(src) % 16 || reinterpret_cast<uintptr_t>(dst) % 16) return CT_E_INVALID;
  if (bytes == 0) return CT_OK;
  const int64_t n16 = bytes / 16;
  k_copy<<<blocks_for(n16, kB * 4, 16384), kB, 0, reinterpret_cast<hipStream_t>(stream)>>>(
      static_cast<const uint4*>(src), static_cast<uint4*>(dst), n16);
  return done();
}

}  // extern "C"

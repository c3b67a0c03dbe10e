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

// G lanes read one line of 16*G bytes; XOR of the line goes to out[i].  A group takes U keys per
// round and issues all U line loads before it reduces any, so each lane has U independent
// 16-byte loads in flight (the container kernels keep up to 8 bucket loads in flight per lane).
// CAS: one 64-bit compare-and-swap on the line's first word; STORE: then an 8-byte store to the
// word after it (an insert's claim and value store into one slot).
template <int G, bool CAS, bool STORE = false>
__global__ __launch_bounds__(kB) void k_gather(uint4* __restrict__ lines, uint64_t nlines,
                                               const uint64_t* __restrict__ keys, int64_t n,
                                               uint64_t* __restrict__ out) {
  constexpr int U = 4;
  const int sub = threadIdx.x % G;
  const int64_t ng = (int64_t)gridDim.x * (kB / G);
  const int64_t rounds = (n + ng * U - 1) / (ng * U);
  for (int64_t r = 0; r < rounds; ++r) {
    const int64_t i0 = r * ng * U + (int64_t)blockIdx.x * (kB / G) + threadIdx.x / G;
    uint64_t key[U], line[U];
    uint4 w[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = min(i0 + u * ng, n - 1);   // clamped: loads are unconditional
      key[u] = keys[i];
      line[u] = __umul64hi(fmix64(key[u]), nlines);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) w[u] = lines[line[u] * G + sub];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = i0 + u * ng;
      uint64_t x = ((uint64_t)w[u].y << 32 | w[u].x) ^ ((uint64_t)w[u].w << 32 | w[u].z);
      for (int off = 1; off < G; off <<= 1) x ^= __shfl_xor(x, off, 64);
      if (sub == 0 && i < n) {
        if (CAS) {
          uint64_t* word = reinterpret_cast<uint64_t*>(&lines[line[u] * G]);
          uint64_t expected = (uint64_t)w[u].y << 32 | w[u].x;
          cas64(word, expected, expected ^ key[u]);
          x ^= expected;
          if (STORE) word[1] = x;
        }
        out[i] = x;
      }
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

// Stream copy: each thread moves U 16-byte words per round, all U loads issued before the stores
// (whole rounds take no bounds tests; the ragged last round does).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kB) void k_copy(const u32x4* __restrict__ src, u32x4* __restrict__ dst,
                                             int64_t n16) {
  constexpr int U = 8;
  const int64_t span = (int64_t)gridDim.x * kB * U;
  int64_t i = (int64_t)blockIdx.x * kB * U + threadIdx.x;
  for (; i + (U - 1) * kB < n16; i += span) {
    u32x4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = __builtin_nontemporal_load(&src[i + u * kB]);
#pragma unroll
    for (int u = 0; u < U; ++u) __builtin_nontemporal_store(v[u], &dst[i + u * kB]);
  }
  for (int u = 0; u < U; ++u)
    if (i + u * kB < n16) dst[i + u * kB] = src[i + u * kB];
}

int blocks_for(int64_t items, int per_block, int cap) {
  const int64_t b = (items + per_block - 1) / per_block;
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, cap));
}

ct_status done() { return hipGetLastError() == hipSuccess ? CT_OK : CT_E_HIP; }

template <bool CAS, bool STORE = false>
ct_status gather(void* lines, int64_t nlines, int32_t line_bytes, const uint64_t* keys, int64_t n,
                 uint64_t* out, void* stream) {
  if (!lines || nlines <= 0 || n < 0 || (n > 0 && (!keys || !out))) return CT_E_INVALID;
  if (line_bytes != 64 && line_bytes != 128) return CT_E_INVALID;
  if (reinterpret_cast<uintptr_t>(lines) % 128) return CT_E_INVALID;
  if (n == 0) return CT_OK;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  uint4* L = static_cast<uint4*>(lines);
  if (line_bytes == 128)
    k_gather<8, CAS, STORE><<<blocks_for(n, kB / 8, 16384), kB, 0, s>>>(L, (uint64_t)nlines, keys, n, out);
  else
    k_gather<4, CAS, STORE><<<blocks_for(n, kB / 4, 16384), kB, 0, s>>>(L, (uint64_t)nlines, keys, n, out);
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

ct_status ctr_gather_cas_store(void* lines, int64_t nlines, int32_t line_bytes,
                               const uint64_t* keys, int64_t n, uint64_t* out, void* stream) {
  return gather<true, true>(lines, nlines, line_bytes, keys, n, out, stream);
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
  k_copy<<<blocks_for(n16, kB * 8, 8192), kB, 0, reinterpret_cast<hipStream_t>(stream)>>>(
      static_cast<const u32x4*>(src), static_cast<u32x4*>(dst), n16);
  return done();
}

}  // extern "C"

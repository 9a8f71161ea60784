// Device helpers shared by the libskew kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace skew {

constexpr int kWave = 64;

// Offset of the per-call error flag inside every workspace (first 256 bytes).
constexpr size_t kFlagBytes = 256;

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// Four int32 keys, loaded as one 16-byte vector.
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));

// Streaming 16-byte load that should not displace the dimension data from L2.
__device__ __forceinline__ i32x4 load_stream4(const i32x4 *p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ int32_t load_stream1(const int32_t *p) { return __builtin_nontemporal_load(p); }

__device__ __forceinline__ void store_stream4(i32x4 *p, i32x4 v) { __builtin_nontemporal_store(v, p); }

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__device__ __forceinline__ void lds_add_u64(uint64_t *p, uint64_t v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void lds_add_u32(uint32_t *p, uint32_t v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void global_add_u64(uint64_t *p, uint64_t v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void global_add_u32(uint32_t *p, uint32_t v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Split of an int32 column at `p` (4-byte aligned) into a scalar head that
// reaches 16-byte alignment, a body of int4 vectors, and a scalar tail.
struct Split4 {
  int64_t head;  // elements [0, head) are scalar
  int64_t nvec;  // vectors cover [head, head + 4 * nvec)
  int64_t tail;  // first scalar element after the body
};

__device__ __forceinline__ Split4 split4(const void *p, int64_t n) {
  Split4 s;
  const uint64_t mis = ((uint64_t)(uintptr_t)p & 15u) >> 2;  // 0..3 elements past alignment
  s.head = mis ? (4 - (int64_t)mis) : 0;
  if (s.head > n) s.head = n;
  s.nvec = (n - s.head) >> 2;
  s.tail = s.head + 4 * s.nvec;
  return s;
}

}  // namespace skew

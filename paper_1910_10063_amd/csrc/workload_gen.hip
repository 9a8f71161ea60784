// Device half of the seeded workload generator (inputs only; holds none of the
// method's arithmetic).  Same definitions as the host half in workload.py:
//   x(seed, j) = splitmix64(seed + (j + 1) * 0x9E3779B97F4A7C15)
//   Zipf rank  = smallest r with cdf[r] > (x >> 11) * 2^-53   (cdf uploaded from the host)
//   uniform    = lo + (((x >> 32) * (hi - lo + 1)) >> 32)
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t draw(uint64_t seed, uint64_t j) {
  return mix64(seed + (j + 1) * 0x9E3779B97F4A7C15ull);
}

__global__ void zipf_keys_kernel(uint64_t seed, const double* __restrict__ cdf, int32_t n_ranks,
                                 const int32_t* __restrict__ pi, int32_t* __restrict__ out,
                                 int64_t n, int64_t start) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const uint64_t x = draw(seed, (uint64_t)(start + i));
    const double u = (double)(x >> 11) * 0x1.0p-53;
    int32_t lo = 0, hi = n_ranks;  // first index with cdf > u, cdf[n_ranks-1] == 1.0
    while (lo < hi) {
      const int32_t mid = lo + ((hi - lo) >> 1);
      if (cdf[mid] > u) hi = mid; else lo = mid + 1;
    }
    out[i] = pi[lo < n_ranks ? lo : n_ranks - 1];
  }
}

__global__ void uniform_kernel(uint64_t seed, int64_t lo, uint64_t range, int32_t* __restrict__ out,
                               int64_t n, int64_t start) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const uint64_t x = draw(seed, (uint64_t)(start + i));
    out[i] = (int32_t)(lo + (int64_t)(((x >> 32) * range) >> 32));
  }
}

int grid_for(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (int)g;
}

}  // namespace

extern "C" int skewgen_fact_keys(uint64_t seed, const double* cdf, int32_t n_ranks, const int32_t* pi,
                                 int32_t* out, int64_t n, int64_t start, void* stream) {
  if (n < 0 || start < 0 || n_ranks < 1 || !cdf || !pi || (n > 0 && !out)) return -1;
  if (n == 0) return 0;
  hipLaunchKernelGGL(zipf_keys_kernel, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, seed, cdf,
                     n_ranks, pi, out, n, start);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

extern "C" int skewgen_uniform_i32(uint64_t seed, int64_t lo, int64_t hi, int32_t* out, int64_t n,
                                   int64_t start, void* stream) {
  const int64_t range = hi - lo + 1;
  if (n < 0 || start < 0 || range < 1 || range > (int64_t)1 << 32 || lo < INT32_MIN || hi > INT32_MAX ||
      (n > 0 && !out))
    return -1;
  if (n == 0) return 0;
  hipLaunchKernelGGL(uniform_kernel, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, seed, lo,
                     (uint64_t)range, out, n, start);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

// Read-bandwidth probe: one pass over a device buffer with 16-byte
// non-temporal loads, reduced to a 64-bit sum so that no load can be
// dropped.  It measures the HBM read rate a streaming kernel reaches on this
// device, the practical ceiling beside the 8 TB/s peak for kernels that
// mostly read (pass 1 of the partitioned join reads 4 bytes per key and
// writes 4 bytes per cold key).
#include "device_common.h"
#include "kernels.h"

namespace skew {
namespace {

constexpr int kProbeThreads = 512;
constexpr int kProbeVecs = 2;  // 16-byte loads per thread per half and step

__device__ __forceinline__ uint64_t word_sum(i32x4 x) {
  return (uint64_t)(uint32_t)x.x + (uint32_t)x.y + (uint64_t)(uint32_t)x.z + (uint32_t)x.w;
}

// The buffer is read as two halves side by side: workgroup b reads the same
// contiguous range of both, so two streams far apart in memory are in flight
// (about 7 % faster on this device than one stream per workgroup).
__global__ __launch_bounds__(kProbeThreads) void stream_probe_kernel(const i32x4 *__restrict__ v, int64_t nvec,
                                                                     unsigned long long *__restrict__ out) {
  const int64_t half = nvec / 2;
  const i32x4 *a = v, *c = v + half;
  const int64_t per = (half + gridDim.x - 1) / gridDim.x;
  const int64_t b = (int64_t)blockIdx.x * per < half ? (int64_t)blockIdx.x * per : half;
  const int64_t e = b + per < half ? b + per : half;
  const int64_t tile = (int64_t)kProbeVecs * blockDim.x;
  uint64_t s = 0;
  int64_t base = b;
  for (; base + tile <= e; base += tile) {
    i32x4 x[kProbeVecs], y[kProbeVecs];
#pragma unroll
    for (int u = 0; u < kProbeVecs; ++u) {
      x[u] = load_stream4(a + base + u * blockDim.x + threadIdx.x);
      y[u] = load_stream4(c + base + u * blockDim.x + threadIdx.x);
    }
#pragma unroll
    for (int u = 0; u < kProbeVecs; ++u) s += word_sum(x[u]) + word_sum(y[u]);
  }
  for (int64_t i = base + threadIdx.x; i < e; i += blockDim.x) s += word_sum(load_stream4(a + i)) + word_sum(load_stream4(c + i));
  if (blockIdx.x == 0)  // the odd vector
    for (int64_t i = 2 * half + threadIdx.x; i < nvec; i += blockDim.x) s += word_sum(load_stream4(v + i));
  s = wave_sum_u64(s);
  if (lane_id() == 0) atomicAdd(out, (unsigned long long)s);
}

}  // namespace

hipError_t launch_stream_probe(const void *buf, size_t bytes, uint64_t *out_sum, const DeviceInfo &dev,
                               hipStream_t s) {
  hipError_t e = hipMemsetAsync(out_sum, 0, 8, s);
  if (e != hipSuccess || bytes == 0) return e;
  const int64_t nvec = (int64_t)(bytes / 16);
  int64_t grid = (nvec / 2 + kProbeThreads - 1) / kProbeThreads;
  const int64_t cap = (int64_t)dev.cu_count * 2;
  if (grid > cap) grid = cap;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(stream_probe_kernel, dim3((int)grid), dim3(kProbeThreads), 0, s,
                     reinterpret_cast<const i32x4 *>(buf), nvec, reinterpret_cast<unsigned long long *>(out_sum));
  return hipGetLastError();
}

}  // namespace skew

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

constexpr int kProbeThreads = 256;
constexpr int kProbeVecs = 4;  // 16-byte loads in flight per thread

__global__ __launch_bounds__(kProbeThreads) void stream_probe_kernel(const i32x4 *__restrict__ v, int64_t nvec,
                                                                     unsigned long long *__restrict__ out) {
  const int64_t T = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t s = 0;
  for (; i + (kProbeVecs - 1) * T < nvec; i += kProbeVecs * T) {
    i32x4 x[kProbeVecs];
#pragma unroll
    for (int u = 0; u < kProbeVecs; ++u) x[u] = load_stream4(v + i + u * T);
#pragma unroll
    for (int u = 0; u < kProbeVecs; ++u)
      s += (uint64_t)(uint32_t)x[u].x + (uint32_t)x[u].y + (uint64_t)(uint32_t)x[u].z + (uint32_t)x[u].w;
  }
  for (; i < nvec; i += T) {
    const i32x4 x = load_stream4(v + i);
    s += (uint64_t)(uint32_t)x.x + (uint32_t)x.y + (uint64_t)(uint32_t)x.z + (uint32_t)x.w;
  }
  s = wave_sum_u64(s);
  if (lane_id() == 0) atomicAdd(out, (unsigned long long)s);
}

}  // namespace

hipError_t launch_stream_probe(const void *buf, size_t bytes, uint64_t *out_sum, const DeviceInfo &dev,
                               hipStream_t s) {
  hipError_t e = hipMemsetAsync(out_sum, 0, 8, s);
  if (e != hipSuccess || bytes == 0) return e;
  const int64_t nvec = (int64_t)(bytes / 16);
  int64_t grid = (nvec + kProbeThreads - 1) / kProbeThreads;
  const int64_t cap = (int64_t)dev.cu_count * 8;
  if (grid > cap) grid = cap;
  hipLaunchKernelGGL(stream_probe_kernel, dim3((int)grid), dim3(kProbeThreads), 0, s,
                     reinterpret_cast<const i32x4 *>(buf), nvec, reinterpret_cast<unsigned long long *>(out_sum));
  return hipGetLastError();
}

}  // namespace skew

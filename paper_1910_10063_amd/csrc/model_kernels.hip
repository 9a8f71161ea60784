// Stack-distance cache model of Section 3.3 on the device: the access
// frequency of every cache line for a layout (Section 3.3: with the
// frequency-ordered layout a line's frequency is the sum of the v largest
// value frequencies; with the identity layout the v keys stored in it), the
// lines sorted by frequency, and one thread per line evaluating the model with
// prefix sums, so that each step of the search for K_i costs O(log L).
#include "kernels.h"
#include "profiler.h"
#include "query_common.h"

namespace skew {
namespace {

__global__ void line_counts_kernel(const uint32_t *__restrict__ counts_by_rank, int32_t n_keys,
                                   const int32_t *__restrict__ rank, int32_t v, int64_t n_lines,
                                   uint32_t *__restrict__ line_counts) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; l < n_lines; l += stride) {
    const int64_t p0 = l * v;
    const int64_t p1 = p0 + v < n_keys ? p0 + v : n_keys;
    uint32_t s = 0;
    for (int64_t p = p0; p < p1; ++p) {
      const uint32_t r = rank ? (uint32_t)rank[p] : (uint32_t)p;
      s += r < (uint32_t)n_keys ? counts_by_rank[r] : 0u;
    }
    line_counts[l] = s;
  }
}

struct ModelLines {
  const uint32_t *c;    // line counts, descending
  const uint32_t *pre;  // pre[j] = c[0] + ... + c[j - 1], j in [0, L]
  int64_t L;
  double F;             // total accesses
};

// Number of lines with count > thr (counts are descending).
__device__ __forceinline__ int64_t lines_above(const ModelLines &m, double thr) {
  int64_t a = 0, z = m.L;  // c[a-1] > thr >= c[z]
  while (a < z) {
    const int64_t mid = (a + z) >> 1;
    if ((double)m.c[mid] > thr) a = mid + 1;
    else z = mid;
  }
  return a;
}

// d(k) for line i: k minus the repeated occurrences k c_j / (F - c_i) - 1 of
// every other line that is expected more than once in k trials.
__device__ __forceinline__ double model_distinct(const ModelLines &m, int64_t i, double ci, double k) {
  const double rest = m.F - ci;
  const int64_t J = lines_above(m, rest / k);
  const bool in = i < J;
  const double sum_c = (double)m.pre[J] - (in ? ci : 0.0);
  const double cnt = (double)J - (in ? 1.0 : 0.0);
  return k - (k * sum_c / rest - cnt);
}

__global__ void model_kernel(ModelLines m, int64_t S, double *__restrict__ contrib) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m.L) return;
  const double ci = (double)m.c[i];
  const double fi = ci / m.F;
  double out = 0.0;
  if (ci > 0.0) {
    const int64_t nonzero = lines_above(m, 0.0);
    if (ci >= m.F || S >= m.L || nonzero - 1 < S) {
      out = fi;  // no other line, or the cache holds every line that occurs
    } else {
      int64_t lo = S, hi = S;
      while (model_distinct(m, i, ci, (double)hi) < (double)S && hi <= ((int64_t)1 << 60)) hi *= 2;
      if (model_distinct(m, i, ci, (double)hi) < (double)S) {
        out = fi;
      } else {
        while (lo < hi) {  // smallest k in [lo, hi] with d(k) >= S
          const int64_t mid = lo + (hi - lo) / 2;
          if (model_distinct(m, i, ci, (double)mid) >= (double)S) hi = mid;
          else lo = mid + 1;
        }
        out = fi * (1.0 - pow(1.0 - fi, (double)lo));
      }
    }
  }
  contrib[i] = out;
}

// Sum of the contributions in a fixed order (one workgroup), so the result
// does not depend on scheduling.
__global__ __launch_bounds__(1024) void model_sum_kernel(const double *__restrict__ contrib, int64_t L,
                                                         double *__restrict__ out) {
  __shared__ double part[1024];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < L; i += blockDim.x) acc += contrib[i];
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = part[0];
}

}  // namespace

size_t model_workspace_bytes(int32_t n_keys, int32_t values_per_line) {
  auto r = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t L = ((size_t)n_keys + values_per_line - 1) / values_per_line;
  const size_t l4 = r(L * 4 + 16);
  return 7 * l4                                     // line counts, sort keys/values x2, sorted, ids
         + r((L + 1) * 4)                           // prefix sums
         + r(L * 8)                                 // contributions
         + r((size_t)256 * 4 * (size_t)sort_tiles((int64_t)L)) + r((size_t)(kScanBlocks + 1) * 4) + r(16) + r(16);
}

hipError_t launch_cache_model(const uint32_t *counts_by_rank, int32_t n_keys, const int32_t *rank,
                              int32_t values_per_line, int64_t cache_lines, void *ws, double *out_hit,
                              const DeviceInfo &dev, hipStream_t s) {
  auto r = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const int64_t L = ((int64_t)n_keys + values_per_line - 1) / values_per_line;
  const size_t l4 = r((size_t)L * 4 + 16);
  char *w = (char *)ws;
  uint32_t *lines = (uint32_t *)w;
  w += l4;
  uint32_t *ka = (uint32_t *)w;
  w += l4;
  uint32_t *kb = (uint32_t *)w;
  w += l4;
  int32_t *va = (int32_t *)w;
  w += l4;
  int32_t *vb = (int32_t *)w;
  w += l4;
  uint32_t *sorted = (uint32_t *)w;
  w += l4;
  int32_t *ids = (int32_t *)w;
  w += l4;
  uint32_t *pre = (uint32_t *)w;
  w += r(((size_t)L + 1) * 4);
  double *contrib = (double *)w;
  w += r((size_t)L * 8);
  uint32_t *digit_hist = (uint32_t *)w;
  w += r((size_t)256 * 4 * (size_t)sort_tiles(L));
  uint32_t *scan = (uint32_t *)w;
  w += r((size_t)(kScanBlocks + 1) * 4);
  uint32_t *total = (uint32_t *)w;
  w += r(16);
  double *hit = (double *)w;

  StageTimer st = stage_begin("model_lines", s);
  const int64_t lgrid = (L + 255) / 256 < (int64_t)dev.cu_count * 16 ? (L + 255) / 256 : (int64_t)dev.cu_count * 16;
  hipLaunchKernelGGL(line_counts_kernel, dim3((int)lgrid), dim3(256), 0, s, counts_by_rank, n_keys, rank,
                     values_per_line, L, lines);
  hipError_t e = hipGetLastError();
  // descending line counts (counts < 2^32: all four digit passes)
  if (e == hipSuccess)
    e = launch_rank_sort(lines, (int32_t)L, (int64_t)0xFFFFFFFFLL, ids, sorted, ka, kb, va, vb, digit_hist, scan, s);
  if (e == hipSuccess) e = hipMemcpyAsync(pre, sorted, (size_t)L * 4, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = launch_exclusive_scan(pre, L, total, scan, s);
  if (e == hipSuccess) e = hipMemcpyAsync(pre + L, total, 4, hipMemcpyDeviceToDevice, s);
  stage_end(st, s);
  if (e != hipSuccess) return e;
  // F is needed on the host side of the launch: read it (the call waits anyway)
  uint32_t F = 0;
  e = hipMemcpyAsync(&F, total, 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  if (F == 0) {
    *out_hit = 0.0;
    return hipSuccess;
  }
  ModelLines m{sorted, pre, L, (double)F};
  st = stage_begin("model_lines_eval", s);
  hipLaunchKernelGGL(model_kernel, dim3((int)((L + 255) / 256)), dim3(256), 0, s, m, cache_lines, contrib);
  e = hipGetLastError();
  stage_end(st, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(model_sum_kernel, dim3(1), dim3(1024), 0, s, contrib, L, hit);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(out_hit, hit, 8, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e;
}

}  // namespace skew

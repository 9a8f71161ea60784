// Prefix sums and cold-item partitioning shared by the layout build and the
// partitioned queries.
#include "kernels.h"
#include "query_common.h"

namespace skew {
namespace {

// ---------------------------------------------------------------------------
// Exclusive prefix sum of `n` u32 values in place, one workgroup of 1024
// threads walking the array in chunks of 8192; `total` (nullable) receives
// the sum of all values.
// ---------------------------------------------------------------------------
constexpr int kScanThreads = 1024;
constexpr int kScanItems = 8;

__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t x) {
  const int lane = lane_id();
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, kWave);
    if (lane >= o) x += y;
  }
  return x;
}

__global__ __launch_bounds__(kScanThreads) void exclusive_scan_kernel(uint32_t *__restrict__ a, int64_t n,
                                                                      uint32_t *__restrict__ total) {
  __shared__ uint32_t wave_off[kScanThreads / kWave];
  __shared__ uint32_t chunk_total;
  const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
  uint32_t carry = 0;
  for (int64_t base = 0; base < n; base += (int64_t)kScanThreads * kScanItems) {
    const int64_t i0 = base + (int64_t)tid * kScanItems;
    uint32_t v[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
      v[j] = i0 + j < n ? a[i0 + j] : 0u;
      s += v[j];
    }
    const uint32_t incl = wave_inclusive_scan(s);
    if (lane == kWave - 1) wave_off[wave] = incl;
    __syncthreads();
    if (wave == 0) {
      const uint32_t ws = lane < kScanThreads / kWave ? wave_off[lane] : 0u;
      const uint32_t wi = wave_inclusive_scan(ws);
      if (lane < kScanThreads / kWave) wave_off[lane] = wi - ws;
      if (lane == kScanThreads / kWave - 1) chunk_total = wi;
    }
    __syncthreads();
    uint32_t run = carry + wave_off[wave] + (incl - s);
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
      if (i0 + j < n) a[i0 + j] = run;
      run += v[j];
    }
    carry += chunk_total;
    __syncthreads();
  }
  if (total && tid == 0) *total = carry;
}

// ---------------------------------------------------------------------------
// Slice plan, step 1: one wave per slice turns the slice's row of per-block
// counts hist[p][0..B) into exclusive prefixes and writes the row total.
// ---------------------------------------------------------------------------
constexpr int kRowScanThreads = 1024;

__global__ __launch_bounds__(kRowScanThreads) void row_scan_kernel(uint32_t *__restrict__ hist, int32_t P, int32_t B,
                                                                   uint32_t *__restrict__ row_total) {
  const int p = blockIdx.x * (kRowScanThreads / kWave) + threadIdx.x / kWave;
  if (p >= P) return;
  uint32_t *row = hist + (int64_t)p * B;
  uint32_t carry = 0;
  for (int b0 = 0; b0 < B; b0 += kWave) {
    const int b = b0 + lane_id();
    const uint32_t v = b < B ? row[b] : 0u;
    const uint32_t incl = wave_inclusive_scan(v);
    if (b < B) row[b] = carry + incl - v;
    carry += __shfl(incl, kWave - 1, kWave);
  }
  if (lane_id() == 0) row_total[p] = carry;
}

// ---------------------------------------------------------------------------
// Slice plan, step 2 (one workgroup, P <= kMaxSlices): the first item of every
// slice (exclusive scan of the row totals) and the total.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kMaxSlices) void slice_plan_kernel(const uint32_t *__restrict__ row_total, int32_t P,
                                                                uint32_t *__restrict__ total,
                                                                uint32_t *__restrict__ slice_off) {
  __shared__ uint32_t wave_off[kMaxSlices / kWave];
  const int p = threadIdx.x, lane = lane_id(), wave = p / kWave;
  const uint32_t cnt = p < P ? row_total[p] : 0u;
  const uint32_t ic = wave_inclusive_scan(cnt);
  if (lane == kWave - 1) wave_off[wave] = ic;
  __syncthreads();
  if (wave == 0) {
    const uint32_t wc = lane < kMaxSlices / kWave ? wave_off[lane] : 0u;
    const uint32_t xc = wave_inclusive_scan(wc);
    if (lane < kMaxSlices / kWave) wave_off[lane] = xc - wc;
  }
  __syncthreads();
  const uint32_t first_item = wave_off[wave] + ic - cnt;
  if (p < P) slice_off[p] = first_item;
  if (p == P - 1) {
    slice_off[P] = first_item + cnt;
    *total = first_item + cnt;
  }
}

// ---------------------------------------------------------------------------
// Scatter: block b moves the cold items of its segment to their slice-order
// positions, as 2-byte offsets inside their slice ((k - t) & (W - 1)) plus the
// value when there is one.  Items are first sorted by slice inside LDS, one
// tile at a time, so that consecutive lanes write consecutive slots.
// ---------------------------------------------------------------------------
constexpr int kScatterThreads = 1024;
constexpr int kScatterVecs = 4;                          // 16-byte loads per thread per tile
constexpr int kScatterPer = 4 * kScatterVecs;            // items per thread per tile
constexpr int kScatterTile = kScatterThreads * kScatterPer;

size_t scatter_lds_bytes(bool pairs) { return (size_t)kScatterTile * 4 * (pairs ? 2 : 1); }

template <bool PAIRS>
__global__ __launch_bounds__(kScatterThreads) void scatter_kernel(
    const int32_t *__restrict__ seg_keys, const int32_t *__restrict__ seg_vals, int64_t seg_cap,
    const uint32_t *__restrict__ seg_count, const uint32_t *__restrict__ hist, const uint32_t *__restrict__ slice_off,
    int32_t P, int32_t t, int32_t wshift, uint16_t *__restrict__ out_local, int32_t *__restrict__ out_vals) {
  __shared__ uint32_t run[kMaxSlices];    // next global slot of every slice for this block
  __shared__ uint32_t start[kMaxSlices];  // tile histogram, then first local slot of every slice
  __shared__ uint32_t wave_off[kScatterThreads / kWave];
  extern __shared__ __align__(16) unsigned char smem[];
  int32_t *skey = reinterpret_cast<int32_t *>(smem);
  int32_t *sval = skey + kScatterTile;  // PAIRS only
  const int b = blockIdx.x, B = gridDim.x, tid = threadIdx.x;
  for (int p = tid; p < P; p += blockDim.x) run[p] = slice_off[p] + hist[(int64_t)p * B + b];
  const uint32_t cnt = seg_count[b];
  // segments start 16-byte aligned and hold a multiple of 4 slots, so every
  // vector that starts below cnt lies inside the segment
  const i32x4 *sk = reinterpret_cast<const i32x4 *>(seg_keys + (int64_t)b * seg_cap);
  const i32x4 *sv = reinterpret_cast<const i32x4 *>(PAIRS ? seg_vals + (int64_t)b * seg_cap : seg_keys);
  const uint32_t wmask = (1u << wshift) - 1u;
  auto slice_of = [&](int32_t k) -> uint32_t {
    const uint32_t p = (uint32_t)(k - t) >> wshift;
    return p < (uint32_t)P ? p : (uint32_t)P - 1;  // pass 1 only writes ids in [t, t + P * W)
  };
  // The next tile is loaded into registers while the current tile is sorted
  // and written.
  i32x4 k[kScatterVecs], v[kScatterVecs], kn[kScatterVecs], vn[kScatterVecs];
  auto load_tile = [&](i32x4(&kk)[kScatterVecs], i32x4(&vv)[kScatterVecs], uint32_t base) {
#pragma unroll
    for (int u = 0; u < kScatterVecs; ++u) {
      const uint32_t vi = base / 4 + (uint32_t)u * kScatterThreads + tid;
      const bool ok = 4 * vi < cnt;
      kk[u] = ok ? load_stream4(sk + vi) : i32x4{0, 0, 0, 0};
      if (PAIRS) vv[u] = ok ? load_stream4(sv + vi) : i32x4{0, 0, 0, 0};
    }
  };
  if (cnt) load_tile(k, v, 0);
  for (uint32_t base = 0; base < cnt; base += kScatterTile) {
    const uint32_t n = cnt - base < (uint32_t)kScatterTile ? cnt - base : (uint32_t)kScatterTile;
    for (int p = tid; p < P; p += blockDim.x) start[p] = 0;
    __syncthreads();
    uint32_t rk[kScatterPer];
#pragma unroll
    for (int u = 0; u < kScatterVecs; ++u) {
      const int32_t kv[4] = {k[u].x, k[u].y, k[u].z, k[u].w};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const uint32_t i = 4 * ((uint32_t)u * kScatterThreads + tid) + j;  // item within the tile
        rk[4 * u + j] = i < n ? atomicAdd(&start[slice_of(kv[j])], 1u) : 0u;  // rank among the tile's items of the slice
      }
    }
    if (base + kScatterTile < cnt) load_tile(kn, vn, base + kScatterTile);
    __syncthreads();
    // exclusive scan of the tile histogram (P <= 1024 entries, one per thread)
    const uint32_t c = tid < P ? start[tid] : 0u;
    uint32_t incl = c;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const uint32_t y = __shfl_up(incl, o, kWave);
      if (lane_id() >= o) incl += y;
    }
    if (lane_id() == kWave - 1) wave_off[tid / kWave] = incl;
    __syncthreads();
    if (tid < kWave) {
      const uint32_t ws = tid < kScatterThreads / kWave ? wave_off[tid] : 0u;
      uint32_t wi = ws;
#pragma unroll
      for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t y = __shfl_up(wi, o, kWave);
        if (lane_id() >= o) wi += y;
      }
      if (tid < kScatterThreads / kWave) wave_off[tid] = wi - ws;
    }
    __syncthreads();
    if (tid < P) start[tid] = wave_off[tid / kWave] + incl - c;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kScatterVecs; ++u) {
      const int32_t kv[4] = {k[u].x, k[u].y, k[u].z, k[u].w};
      const int32_t vv[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const uint32_t i = 4 * ((uint32_t)u * kScatterThreads + tid) + j;
        if (i < n) {
          const uint32_t pos = start[slice_of(kv[j])] + rk[4 * u + j];
          skey[pos] = kv[j];
          if (PAIRS) sval[pos] = vv[j];
        }
      }
    }
    __syncthreads();
    for (uint32_t j = tid; j < n; j += kScatterThreads) {
      const int32_t kk = skey[j];
      const uint32_t p = slice_of(kk);
      const uint32_t g = run[p] + (j - start[p]);
      out_local[g] = (uint16_t)((uint32_t)(kk - t) & wmask);
      if (PAIRS) out_vals[g] = sval[j];
    }
    __syncthreads();
    if (tid < P) run[tid] += c;
#pragma unroll
    for (int u = 0; u < kScatterVecs; ++u) {
      k[u] = kn[u];
      if (PAIRS) v[u] = vn[u];
    }
  }
}

}  // namespace

hipError_t launch_exclusive_scan(uint32_t *a, int64_t n, uint32_t *total, hipStream_t s) {
  hipLaunchKernelGGL(exclusive_scan_kernel, dim3(1), dim3(kScanThreads), 0, s, a, n, total);
  return hipGetLastError();
}

hipError_t launch_partition_plan(const SliceTables &tab, int32_t P, int32_t B, hipStream_t s) {
  constexpr int per_block = kRowScanThreads / kWave;
  hipLaunchKernelGGL(row_scan_kernel, dim3((P + per_block - 1) / per_block), dim3(kRowScanThreads), 0, s, tab.hist, P, B,
                     tab.row_total);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(slice_plan_kernel, dim3(1), dim3(kMaxSlices), 0, s, tab.row_total, P, tab.total, tab.slice_off);
  return hipGetLastError();
}

hipError_t launch_partition_scatter(const SliceTables &tab, int32_t P, int32_t B, const int32_t *seg_keys,
                                    const int32_t *seg_vals, int64_t seg_cap, int32_t t, int32_t wshift,
                                    uint16_t *out_local, int32_t *out_vals, hipStream_t s) {
  if (seg_vals) {
    const size_t lds = scatter_lds_bytes(true);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(scatter_kernel<true>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(scatter_kernel<true>, dim3(B), dim3(kScatterThreads), lds, s, seg_keys, seg_vals, seg_cap,
                       tab.seg_count, tab.hist, tab.slice_off, P, t, wshift, out_local, out_vals);
  } else {
    const size_t lds = scatter_lds_bytes(false);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(scatter_kernel<false>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(scatter_kernel<false>, dim3(B), dim3(kScatterThreads), lds, s, seg_keys, seg_vals, seg_cap,
                       tab.seg_count, tab.hist, tab.slice_off, P, t, wshift, out_local, out_vals);
  }
  return hipGetLastError();
}

}  // namespace skew

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
constexpr int kHistSliceShift = 15;  // 32768 counters per LDS slice of the histogram
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

// Exclusive scan of a[0, n) in place starting from `carry`, by one workgroup;
// returns the sum of the range (to thread 0).
__device__ __forceinline__ uint32_t scan_range(uint32_t *__restrict__ a, int64_t n, uint32_t carry) {
  __shared__ uint32_t wave_off[kScanThreads / kWave];
  __shared__ uint32_t chunk_total;
  const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
  uint32_t sum = 0;
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
    uint32_t run = carry + sum + wave_off[wave] + (incl - s);
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
      if (i0 + j < n) a[i0 + j] = run;
      run += v[j];
    }
    sum += chunk_total;
    __syncthreads();
  }
  return sum;
}

__global__ __launch_bounds__(kScanThreads) void exclusive_scan_kernel(uint32_t *__restrict__ a, int64_t n,
                                                                      uint32_t *__restrict__ total) {
  const uint32_t sum = scan_range(a, n, 0u);
  if (total && threadIdx.x == 0) *total = sum;
}

// Multi-workgroup form: workgroup b owns a[b * per, (b + 1) * per).
__global__ __launch_bounds__(kScanThreads) void chunk_sum_kernel(const uint32_t *__restrict__ a, int64_t n,
                                                                 int64_t per, uint32_t *__restrict__ sums) {
  __shared__ uint32_t part[kScanThreads / kWave];
  const int64_t lo = (int64_t)blockIdx.x * per;
  const int64_t hi = lo + per < n ? lo + per : n;
  uint32_t s = 0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) s += a[i];
  s = wave_sum_u32(s);
  if (lane_id() == 0) part[threadIdx.x / kWave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int w = 0; w < kScanThreads / kWave; ++w) t += part[w];
    sums[blockIdx.x] = t;
  }
}

__global__ __launch_bounds__(kScanThreads) void chunk_scan_kernel(uint32_t *__restrict__ a, int64_t n, int64_t per,
                                                                  const uint32_t *__restrict__ offsets) {
  const int64_t lo = (int64_t)blockIdx.x * per;
  const int64_t hi = lo + per < n ? lo + per : n;
  (void)scan_range(a + lo, hi - lo, offsets[blockIdx.x]);
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
// value when there is one; a narrow record (group << 12 | value, t = 0) moves
// as one word, offset << 12 | value.  Items are first sorted by slice inside
// LDS, one tile at a time, so that consecutive lanes write consecutive slots.
// ---------------------------------------------------------------------------
constexpr int kScatterThreads = 1024;
constexpr int kScatterVecs = 4;                          // 16-byte loads per thread per tile
constexpr int kScatterPer = 4 * kScatterVecs;            // items per thread per tile
constexpr int kScatterTile = kScatterThreads * kScatterPer;

size_t scatter_lds_bytes(bool pairs) { return (size_t)kScatterTile * 4 * (pairs ? 2 : 1); }

template <bool PAIRS, bool NARROW = false, bool COMBINE0 = false>
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
  // With COMBINE0, when this block's items of slice 0 (the row scan left exclusive prefixes over the blocks)
  // are half of its segment or more, the lanes of a load that fall into slice 0 take their ranks together.
  bool combine0 = false;
  if (COMBINE0) {
    const uint32_t n0 = (b + 1 < B ? hist[b + 1] : slice_off[1] - slice_off[0]) - hist[b];
    combine0 = 2ull * n0 >= (uint64_t)cnt && cnt > 0;
  }
  // segments start 16-byte aligned and hold a multiple of 4 slots, so every
  // vector that starts below cnt lies inside the segment
  const i32x4 *sk = reinterpret_cast<const i32x4 *>(seg_keys + (int64_t)b * seg_cap);
  const i32x4 *sv = reinterpret_cast<const i32x4 *>(PAIRS ? seg_vals + (int64_t)b * seg_cap : seg_keys);
  const uint32_t wmask = (1u << wshift) - 1u;
  auto key_of = [&](int32_t k) -> int32_t { return NARROW ? (int32_t)((uint32_t)k >> kGroupNarrowShift) : k; };
  auto slice_of = [&](int32_t k) -> uint32_t {
    const uint32_t p = (uint32_t)(key_of(k) - t) >> wshift;
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
        // rank among the tile's items of the slice; the lanes whose items fall into slice 0 (the densest
        // one on a frequency-ordered layout) take consecutive ranks with one LDS add
        const uint32_t sl = slice_of(kv[j]);
        if (COMBINE0 && combine0) {
          const bool z = i < n && sl == 0;
          const uint64_t mz = __ballot(z);
          uint32_t base0 = 0;
          if (z && lanes_below(mz) == 0) base0 = atomicAdd(&start[0], (uint32_t)__popcll(mz));
          base0 = (uint32_t)__shfl((int)base0, (int)(__ffsll((unsigned long long)mz) - 1) & (kWave - 1), kWave);
          rk[4 * u + j] = z ? base0 + lanes_below(mz) : (i < n ? atomicAdd(&start[sl], 1u) : 0u);
        } else {
          rk[4 * u + j] = i < n ? atomicAdd(&start[sl], 1u) : 0u;
        }
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
      if (NARROW) {
        const uint32_t vmask = (1u << kGroupNarrowShift) - 1u;
        out_vals[g] = (int32_t)((((uint32_t)key_of(kk) & wmask) << kGroupNarrowShift) | ((uint32_t)kk & vmask));
      } else {
        out_local[g] = (uint16_t)((uint32_t)(kk - t) & wmask);
        if (PAIRS) out_vals[g] = sval[j];
      }
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

// ---------------------------------------------------------------------------
// Partitioned key histogram: the frequency count that starts the index build
// (Section 3.1), run as a partitioned aggregation because the hot keys are
// not known yet.  Pass 1 appends every key in [0, n_keys) to its workgroup's
// segment and counts it in its slice (k >> 15); the shared plan and scatter
// above order the keys by slice as 2-byte offsets; pass 3 counts every slice
// in LDS and adds the counts into the histogram.
//
// Large columns first count a sample (their first kHotSample keys) this
// way, take the keys whose sample count is highest (at most kHotMax of them,
// the likely hot keys) into a hash table, and count the rest of the column
// with that table in LDS: a key found there is counted in an LDS counter of
// its slot, and only the others are partitioned.  A key is counted exactly
// once either way, so the counts do not depend on which keys the table holds.
// ---------------------------------------------------------------------------
constexpr int kHistThreads = 1024;
constexpr int kHistVecs = 4;
constexpr int kHotBucketBits = 12;
constexpr int kHotBuckets = 1 << kHotBucketBits;  // 4-slot buckets
constexpr int kHotSlots = 4 * kHotBuckets;         // 16384 slots: keys 64 KB + counters 64 KB of LDS
constexpr int kHotMax = 3 * kHotBuckets;           // keys offered to the table (75 % of the slots)
constexpr int kCountBins = 256;                    // 8 bins per power of two of a count
constexpr int64_t kHotSample = 1LL << 24;          // keys counted before the table is chosen
constexpr int64_t kHotMinFact = 1LL << 26;         // smaller columns skip the table

__device__ __forceinline__ uint32_t hot_bucket(uint32_t k) { return (k * 0x9E3779B1u) >> (32 - kHotBucketBits); }

// Bin of a count c >= 1: floor(log2 c) and the next three bits, so bins rise with c.
__device__ __forceinline__ int count_bin(uint32_t c) {
  const int e = 31 - __clz(c);
  const uint32_t m = e >= 3 ? (c >> (e - 3)) & 7u : (c << (3 - e)) & 7u;
  return e * 8 + (int)m;
}

// f(k, counts[k]) for every k in [0, n_keys): four counts per 16-byte load,
// the last n_keys mod 4 one by one.
template <class F>
__device__ __forceinline__ void for_each_count(const uint32_t *__restrict__ counts, int32_t n_keys, F f) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t nv = n_keys / 4;
  const uint4 *v = reinterpret_cast<const uint4 *>(counts);  // the histogram is 256-byte aligned
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += stride) {
    const uint4 c = v[i];
    f(4 * i, c.x);
    f(4 * i + 1, c.y);
    f(4 * i + 2, c.z);
    f(4 * i + 3, c.w);
  }
  if (blockIdx.x == 0 && threadIdx.x < (unsigned)(n_keys - 4 * nv))
    f(4 * nv + threadIdx.x, counts[4 * nv + threadIdx.x]);
}

// Sample counts below this cannot make a table worth its lookups (12288 keys
// of fewer than 4 sample rows each cover under 0.3 % of a 2^24-key sample).
constexpr uint32_t kHotMinCount = 4;

// Number of keys and their total count per count bin (counts >= kHotMinCount).
__global__ void count_bins_kernel(const uint32_t *__restrict__ counts, int32_t n_keys, uint32_t *__restrict__ bin_n,
                                  unsigned long long *__restrict__ bin_sum) {
  __shared__ uint32_t ln[kCountBins];
  __shared__ unsigned long long ls[kCountBins];
  for (int i = threadIdx.x; i < kCountBins; i += blockDim.x) {
    ln[i] = 0;
    ls[i] = 0;
  }
  __syncthreads();
  for_each_count(counts, n_keys, [&](int64_t, uint32_t c) {
    if (c >= kHotMinCount) {
      const int b = count_bin(c);
      atomicAdd(&ln[b], 1u);
      atomicAdd(&ls[b], (unsigned long long)c);
    }
  });
  __syncthreads();
  for (int i = threadIdx.x; i < kCountBins; i += blockDim.x)
    if (ln[i]) {
      atomicAdd(&bin_n[i], ln[i]);
      atomicAdd(&bin_sum[i], ls[i]);
    }
}

// The lowest bin from which on at most kHotMax keys lie; no bin (kCountBins)
// when those keys cover less than an eighth of the sample, since the table
// would then cost more lookups than it saves.  Clears the key count.
__global__ void pick_hot_kernel(const uint32_t *__restrict__ bin_n, const unsigned long long *__restrict__ bin_sum,
                                uint64_t sample, int32_t *__restrict__ tau, uint32_t *__restrict__ hot_n) {
  if (threadIdx.x != 0) return;
  uint32_t keys = 0;
  unsigned long long cover = 0;
  int b = kCountBins;
  while (b > 0 && keys + bin_n[b - 1] <= (uint32_t)kHotMax) {
    --b;
    keys += bin_n[b];
    cover += bin_sum[b];
  }
  *tau = (keys > 0 && cover * 8 >= sample) ? b : kCountBins;
  *hot_n = 0;
}

__global__ void collect_hot_kernel(const uint32_t *__restrict__ counts, int32_t n_keys, const int32_t *__restrict__ tau,
                                   int32_t *__restrict__ hot_keys, uint32_t *__restrict__ hot_n) {
  const int t = *tau;
  if (t >= kCountBins) return;
  for_each_count(counts, n_keys, [&](int64_t k, uint32_t c) {
    if (c >= kHotMinCount && count_bin(c) >= t) {
      const uint32_t i = atomicAdd(hot_n, 1u);
      if (i < (uint32_t)kHotMax) hot_keys[i] = (int32_t)k;
    }
  });
}

// One workgroup inserts the chosen keys into the 4-slot buckets (a key whose
// bucket is full stays out) and writes the table; every workgroup of the
// split then loads the same table.
__global__ __launch_bounds__(kHistThreads) void hot_table_kernel(const int32_t *__restrict__ hot_keys,
                                                                 const uint32_t *__restrict__ hot_n,
                                                                 int32_t *__restrict__ table) {
  __shared__ int32_t tk[kHotSlots];
  for (int i = threadIdx.x; i < kHotSlots; i += blockDim.x) tk[i] = -1;
  __syncthreads();
  const uint32_t n = *hot_n < (uint32_t)kHotMax ? *hot_n : (uint32_t)kHotMax;
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
    const int32_t k = hot_keys[i];
    const uint32_t b = hot_bucket((uint32_t)k) * 4;
    for (int j = 0; j < 4; ++j)
      if (atomicCAS(&tk[b + j], -1, k) == -1) break;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kHotSlots; i += blockDim.x) table[i] = tk[i];
}

// Per-slot counts of the workgroups, added into the histogram: grid.y cuts
// the workgroups into groups of kReduceRows, each added with one atomic.
constexpr int kReduceRows = 16;

__global__ void hot_reduce_kernel(const uint32_t *__restrict__ partial, int32_t blocks, const int32_t *__restrict__ table,
                                  uint32_t *__restrict__ counts) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= kHotSlots) return;
  const int32_t k = table[s];
  if (k < 0) return;
  const int b0 = blockIdx.y * kReduceRows;
  const int b1 = b0 + kReduceRows < blocks ? b0 + kReduceRows : blocks;
  uint32_t c = 0;
#pragma unroll 8
  for (int b = b0; b < b1; ++b) c += partial[(int64_t)b * kHotSlots + s];
  if (c) global_add_u32(&counts[k], c);
}

// HOT: keys found in the hot table are counted in LDS (partial[block][slot]
// at the end) instead of being partitioned.
template <bool HOT>
__global__ __launch_bounds__(kHistThreads) void hist_split_kernel(const int32_t *__restrict__ keys, int64_t n,
                                                                  int32_t n_keys, int32_t P, int32_t *__restrict__ seg,
                                                                  int64_t seg_cap, uint32_t *__restrict__ seg_count,
                                                                  uint32_t *__restrict__ hist, int32_t *flag,
                                                                  const int32_t *__restrict__ table,
                                                                  const int32_t *__restrict__ tau,
                                                                  uint32_t *__restrict__ partial) {
  __shared__ uint32_t lhist[kMaxSlices + kWave + 1];  // slice counts | per-lane sinks | item count
  extern __shared__ __align__(16) unsigned char smem[];
  int32_t *tkeys = reinterpret_cast<int32_t *>(smem);                  // HOT: [kHotSlots]
  uint32_t *tcnt = reinterpret_cast<uint32_t *>(tkeys + kHotSlots);   // HOT: [kHotSlots + kWave]
  for (int p = threadIdx.x; p < P + kWave + 1; p += blockDim.x) lhist[p] = 0;
  const bool use_hot = HOT && *tau < kCountBins;  // same for every thread
  if (use_hot) {
    for (int i = threadIdx.x; i < kHotSlots; i += blockDim.x) tkeys[i] = table[i];
    for (int i = threadIdx.x; i < kHotSlots + kWave; i += blockDim.x) tcnt[i] = 0;
  }
  __syncthreads();
  ColdSink o;
  o.count = &lhist[P + kWave];
  o.hist = lhist;
  o.t = 0;
  o.wshift = kHistSliceShift;
  o.sink = (uint32_t)P + lane_id();
  const rsrc_t out = record_buffer(seg + (int64_t)blockIdx.x * seg_cap, (uint32_t)seg_cap);
  const uint32_t nk = (uint32_t)n_keys;
  bool bad = false;
  auto put = [&](const uint32_t(&k)[4 * kHistVecs], const bool(&ok)[4 * kHistVecs]) {
    bool in[4 * kHistVecs];
#pragma unroll
    for (int i = 0; i < 4 * kHistVecs; ++i) {
      in[i] = ok[i] && k[i] < nk;
      bad |= ok[i] && k[i] >= nk;
    }
    if (use_hot) {
#pragma unroll
      for (int i = 0; i < 4 * kHistVecs; ++i) {
        const uint32_t b = hot_bucket(k[i]) * 4;
        const i32x4 ks = *reinterpret_cast<const i32x4 *>(tkeys + b);
        const bool h0 = ks.x == (int32_t)k[i], h1 = ks.y == (int32_t)k[i], h2 = ks.z == (int32_t)k[i];
        const bool hit = in[i] && (h0 || h1 || h2 || ks.w == (int32_t)k[i]);
        const uint32_t slot = h0 ? b : (h1 ? b + 1 : (h2 ? b + 2 : b + 3));
        lds_add_u32(&tcnt[hit ? slot : (uint32_t)kHotSlots + lane_id()], 1u);
        in[i] = in[i] && !hit;
      }
    }
    cold_append(o, k, in, [&](int i, int32_t idx) { buffer_store_record((int32_t)k[i], out, idx, 0, 0, 0); });
  };
  const Split4 sp = split4(keys, n);
  {  // scalar head (block 0, lanes 0-2) and tail (last block, lanes 64-66), one slot per lane
    int64_t i = -1;
    if (blockIdx.x == 0 && threadIdx.x < sp.head) i = threadIdx.x;
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x >= kWave && threadIdx.x - kWave < n - sp.tail)
      i = sp.tail + threadIdx.x - kWave;
    uint32_t k1[4 * kHistVecs];
    bool ok1[4 * kHistVecs];
#pragma unroll
    for (int j = 0; j < 4 * kHistVecs; ++j) {
      k1[j] = 0;
      ok1[j] = false;
    }
    k1[0] = i >= 0 ? (uint32_t)keys[i] : 0u;
    ok1[0] = i >= 0;
    put(k1, ok1);
  }
  const i32x4 *vk = reinterpret_cast<const i32x4 *>(keys + sp.head);
  const int64_t per = (sp.nvec + gridDim.x - 1) / gridDim.x;
  const int64_t vb = (int64_t)blockIdx.x * per < sp.nvec ? (int64_t)blockIdx.x * per : sp.nvec;
  const int64_t ve = vb + per < sp.nvec ? vb + per : sp.nvec;
  constexpr int64_t kTile = (int64_t)kHistThreads * kHistVecs;
  auto unpack = [&](const i32x4(&x)[kHistVecs], uint32_t(&k)[4 * kHistVecs]) {
#pragma unroll
    for (int u = 0; u < kHistVecs; ++u) {
      k[4 * u] = (uint32_t)x[u].x, k[4 * u + 1] = (uint32_t)x[u].y;
      k[4 * u + 2] = (uint32_t)x[u].z, k[4 * u + 3] = (uint32_t)x[u].w;
    }
  };
  bool all_ok[4 * kHistVecs];
#pragma unroll
  for (int i = 0; i < 4 * kHistVecs; ++i) all_ok[i] = true;
  auto load_tile = [&](i32x4(&x)[kHistVecs], int64_t base) {
#pragma unroll
    for (int u = 0; u < kHistVecs; ++u) x[u] = load_stream4(vk + base + u * kHistThreads + threadIdx.x);
  };
  const int64_t full_end = vb + ((ve - vb) / kTile) * kTile;
  i32x4 xa[kHistVecs], xb[kHistVecs];
  uint32_t k[4 * kHistVecs];
  int64_t base = vb;
  if (base < full_end) load_tile(xa, base);
  while (base < full_end) {  // unconditional prefetch: the last one re-reads the current tile
    int64_t nxt = base + kTile;
    load_tile(xb, nxt < full_end ? nxt : base);
    unpack(xa, k);
    put(k, all_ok);
    base = nxt;
    if (base >= full_end) break;
    nxt = base + kTile;
    load_tile(xa, nxt < full_end ? nxt : base);
    unpack(xb, k);
    put(k, all_ok);
    base = nxt;
  }
  if (full_end < ve) {
    i32x4 x[kHistVecs];
    bool ok[4 * kHistVecs];
#pragma unroll
    for (int u = 0; u < kHistVecs; ++u) {
      const int64_t vi = full_end + u * kHistThreads + threadIdx.x;
      x[u] = vi < ve ? load_stream4(vk + vi) : i32x4{0, 0, 0, 0};
#pragma unroll
      for (int j = 0; j < 4; ++j) ok[4 * u + j] = vi < ve;
    }
    unpack(x, k);
    put(k, ok);
  }
  if (bad) *flag = 1;
  __syncthreads();
  if (threadIdx.x == 0) seg_count[blockIdx.x] = *o.count < seg_cap ? *o.count : (uint32_t)seg_cap;
  for (int p = threadIdx.x; p < P; p += blockDim.x) hist[(int64_t)p * gridDim.x + blockIdx.x] = lhist[p];
  if (use_hot)
    for (int i = threadIdx.x; i < kHotSlots; i += blockDim.x) partial[(int64_t)blockIdx.x * kHotSlots + i] = tcnt[i];
}

// Pass 3.  Within a wave the value of the first active lane is often the
// slice's dominant key (random key order puts the hottest keys in slices of
// their own): its lanes are added once, by one lane, with the ballot count;
// the others add 1; lanes with nothing to add hit a sink word of their own.
constexpr int kHistSliceVecs = 2;

__device__ __forceinline__ void hist_add(uint32_t *bins, uint32_t v, bool ok) {
  const uint32_t sink = (1u << kHistSliceShift) + lane_id();
  const uint32_t lead = __builtin_amdgcn_readfirstlane(ok ? v : 0xFFFFFFFFu);
  const bool dup = ok && v == lead;
  const uint64_t m = __ballot(dup);
  const bool first = dup && lanes_below(m) == 0;
  const uint32_t addr = !ok ? sink : (dup ? (first ? v : sink) : v);
  const uint32_t inc = !ok ? 0u : (dup ? (first ? (uint32_t)__popcll(m) : 0u) : 1u);
  lds_add_u32(&bins[addr], inc);
}

__global__ __launch_bounds__(kHistThreads) void hist_slice_kernel(const uint16_t *__restrict__ locals,
                                                                  const uint32_t *__restrict__ slice_off, int32_t P,
                                                                  int32_t n_keys, uint32_t *__restrict__ counts) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int32_t W = 1 << kHistSliceShift;
  uint32_t *bins = reinterpret_cast<uint32_t *>(smem);  // [W] counters | [64] sinks
  uint32_t *soff = bins + W + kWave;
  for (int i = threadIdx.x; i < W + kWave; i += blockDim.x) bins[i] = 0;
  for (int p = threadIdx.x; p <= P; p += blockDim.x) soff[p] = slice_off[p];
  __syncthreads();
  uint32_t lo, hi;
  balanced_share(soff, P, (uint32_t)W, blockIdx.x, gridDim.x, &lo, &hi);
  int32_t p = lo < hi ? slice_of_item(soff, P, lo) : P;
  const i32x4 *vl = reinterpret_cast<const i32x4 *>(locals);
  for (uint32_t at = lo; at < hi; ++p) {
    const uint32_t end = soff[p + 1] < hi ? soff[p + 1] : hi;
    if (end <= at) continue;
    const int64_t sbase = (int64_t)p << kHistSliceShift;
    const int32_t slen = (int32_t)((int64_t)n_keys - sbase < W ? (int64_t)n_keys - sbase : W);
    walk_items<8, kHistSliceVecs, kHistThreads, i32x4>(
        at, end, [&](uint32_t i) { lds_add_u32(&bins[locals[i]], 1u); },
        [&](uint32_t vi) { return load_stream4(vl + vi); },
        [&](const i32x4(&x)[kHistSliceVecs], const bool(&valid)[kHistSliceVecs]) {
#pragma unroll
          for (int u = 0; u < kHistSliceVecs; ++u) {
            const uint32_t d[4] = {(uint32_t)x[u].x, (uint32_t)x[u].y, (uint32_t)x[u].z, (uint32_t)x[u].w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              hist_add(bins, d[j] & 0xFFFFu, valid[u]);
              hist_add(bins, d[j] >> 16, valid[u]);
            }
          }
        });
    __syncthreads();
    for (int i = threadIdx.x; i < slen; i += blockDim.x) {
      const uint32_t c = bins[i];
      if (c) {
        global_add_u32(&counts[sbase + i], c);
        bins[i] = 0;
      }
    }
    __syncthreads();
    at = end;
  }
}

}  // namespace

hipError_t launch_exclusive_scan(uint32_t *a, int64_t n, uint32_t *total, uint32_t *scratch, hipStream_t s) {
  // With scratch (kScanBlocks + 1 words): chunk sums, one scan over them, then
  // every chunk scanned from its offset.  Small arrays, or no scratch: one
  // workgroup.
  constexpr int64_t kChunk = (int64_t)kScanThreads * kScanItems;
  if (!scratch || n <= 4 * kChunk) {
    hipLaunchKernelGGL(exclusive_scan_kernel, dim3(1), dim3(kScanThreads), 0, s, a, n, total);
    return hipGetLastError();
  }
  int64_t per = (n + kScanBlocks - 1) / kScanBlocks;
  per = (per + kChunk - 1) / kChunk * kChunk;
  const int blocks = (int)((n + per - 1) / per);
  hipLaunchKernelGGL(chunk_sum_kernel, dim3(blocks), dim3(kScanThreads), 0, s, a, n, per, scratch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(exclusive_scan_kernel, dim3(1), dim3(kScanThreads), 0, s, scratch, (int64_t)blocks, total);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(chunk_scan_kernel, dim3(blocks), dim3(kScanThreads), 0, s, a, n, per, scratch);
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
                                    uint16_t *out_local, int32_t *out_vals, hipStream_t s, bool combine0) {
  auto go = [&](auto kernel, bool pairs) {
    const size_t lds = scatter_lds_bytes(pairs);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
    hipLaunchKernelGGL(kernel, dim3(B), dim3(kScatterThreads), lds, s, seg_keys, seg_vals, seg_cap, tab.seg_count,
                       tab.hist, tab.slice_off, P, t, wshift, out_local, out_vals);
  };
  if (seg_vals) {
    if (combine0) go(scatter_kernel<true, false, true>, true);
    else go(scatter_kernel<true, false, false>, true);
  } else {
    if (combine0) go(scatter_kernel<false, false, true>, false);
    else go(scatter_kernel<false, false, false>, false);
  }
  return hipGetLastError();
}

hipError_t launch_partition_scatter_narrow(const SliceTables &tab, int32_t P, int32_t B, const int32_t *seg_recs,
                                           int64_t seg_cap, int32_t wshift, int32_t *out_items, hipStream_t s,
                                           bool combine0) {
  auto go = [&](auto kernel) {
    const size_t lds = scatter_lds_bytes(false);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
    hipLaunchKernelGGL(kernel, dim3(B), dim3(kScatterThreads), lds, s, seg_recs, nullptr, seg_cap, tab.seg_count,
                       tab.hist, tab.slice_off, P, 0, wshift, nullptr, out_items);
  };
  if (combine0) go(scatter_kernel<false, true, true>);
  else go(scatter_kernel<false, true, false>);
  return hipGetLastError();
}

HistPlan hist_plan(int64_t n_fact, int32_t n_keys, const DeviceInfo &dev) {
  HistPlan pl;
  pl.blocks = dev.cu_count > 0 ? dev.cu_count : 256;
  pl.slices = (int32_t)(((int64_t)n_keys + (1 << kHistSliceShift) - 1) >> kHistSliceShift);
  pl.round = n_fact < kMaxRound ? n_fact : kMaxRound;
  const int64_t nvec = (pl.round + 3) / 4 + 1;
  pl.seg_cap = 4 * ((nvec + pl.blocks - 1) / pl.blocks) + 8;
  return pl;
}

// Hot-table region: count bins, the cut, the chosen keys, the table and the
// per-workgroup slot counts.
static size_t hot_region_bytes(int32_t blocks) {
  auto r = [](size_t x) { return (x + 255) & ~(size_t)255; };
  return r((size_t)kCountBins * 4) + r((size_t)kCountBins * 8) + r(16) + r((size_t)kHotMax * 4) +
         r((size_t)kHotSlots * 4) + r((size_t)blocks * kHotSlots * 4);
}

size_t hist_partition_bytes(const HistPlan &pl) {
  auto r = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const int32_t P = pl.slices > 0 ? pl.slices : 1;
  return r((size_t)pl.blocks * pl.seg_cap * 4) + r((size_t)pl.round * 2 + 16) + r((size_t)P * pl.blocks * 4) +
         r((size_t)P * 4) + r(4) + r((size_t)pl.blocks * 4) + r((size_t)(P + 1) * 4) + hot_region_bytes(pl.blocks);
}

hipError_t launch_histogram_partitioned(const int32_t *keys, int64_t n_fact, int32_t n_keys, uint32_t *counts,
                                        int32_t *flag, void *part_ws, const HistPlan &pl, hipStream_t s) {
  auto r = [](size_t x) { return (x + 255) & ~(size_t)255; };
  char *ws = (char *)part_ws;
  int32_t *seg = (int32_t *)ws;
  ws += r((size_t)pl.blocks * pl.seg_cap * 4);
  uint16_t *items = (uint16_t *)ws;
  ws += r((size_t)pl.round * 2 + 16);
  SliceTables tab;
  tab.hist = (uint32_t *)ws;
  ws += r((size_t)pl.slices * pl.blocks * 4);
  tab.row_total = (uint32_t *)ws;
  ws += r((size_t)pl.slices * 4);
  tab.total = (uint32_t *)ws;
  ws += r(4);
  tab.seg_count = (uint32_t *)ws;
  ws += r((size_t)pl.blocks * 4);
  tab.slice_off = (uint32_t *)ws;
  ws += r((size_t)(pl.slices + 1) * 4);
  uint32_t *bin_n = (uint32_t *)ws;
  ws += r((size_t)kCountBins * 4);
  unsigned long long *bin_sum = (unsigned long long *)ws;
  ws += r((size_t)kCountBins * 8);
  int32_t *tau = (int32_t *)ws;
  uint32_t *hot_n = (uint32_t *)(ws + 4);
  ws += r(16);
  int32_t *hot_keys = (int32_t *)ws;
  ws += r((size_t)kHotMax * 4);
  int32_t *table = (int32_t *)ws;
  ws += r((size_t)kHotSlots * 4);
  uint32_t *partial = (uint32_t *)ws;

  const size_t lds3 = ((size_t)(1 << kHistSliceShift) + kWave + pl.slices + 1) * 4;
  const size_t lds_hot = (size_t)(2 * kHotSlots + kWave) * 4;
  (void)hipFuncSetAttribute(reinterpret_cast<const void *>(hist_slice_kernel),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds3);
  (void)hipFuncSetAttribute(reinterpret_cast<const void *>(hist_split_kernel<true>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_hot);
  // one round of the partitioned count over keys [lo, hi), with or without the hot table
  auto count_rounds = [&](int64_t lo, int64_t hi, bool hot) -> hipError_t {
    for (int64_t off = lo; off < hi; off += pl.round) {
      const int64_t n = hi - off < pl.round ? hi - off : pl.round;
      if (hot)
        hipLaunchKernelGGL(hist_split_kernel<true>, dim3(pl.blocks), dim3(kHistThreads), lds_hot, s, keys + off, n,
                           n_keys, pl.slices, seg, pl.seg_cap, tab.seg_count, tab.hist, flag, table, tau, partial);
      else
        hipLaunchKernelGGL(hist_split_kernel<false>, dim3(pl.blocks), dim3(kHistThreads), 0, s, keys + off, n, n_keys,
                           pl.slices, seg, pl.seg_cap, tab.seg_count, tab.hist, flag, table, tau, partial);
      hipError_t e = hipGetLastError();
      if (e == hipSuccess) e = launch_partition_plan(tab, pl.slices, pl.blocks, s);
      if (e == hipSuccess)
        e = launch_partition_scatter(tab, pl.slices, pl.blocks, seg, nullptr, pl.seg_cap, 0, kHistSliceShift, items,
                                     nullptr, s);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(hist_slice_kernel, dim3(pl.blocks), dim3(kHistThreads), lds3, s, items, tab.slice_off,
                         pl.slices, n_keys, counts);
      e = hipGetLastError();
      if (e == hipSuccess && hot) {
        hipLaunchKernelGGL(hot_reduce_kernel, dim3(kHotSlots / 256, (pl.blocks + kReduceRows - 1) / kReduceRows),
                           dim3(256), 0, s, partial, pl.blocks, table, counts);
        e = hipGetLastError();
      }
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  };
  if (n_fact < kHotMinFact) return count_rounds(0, n_fact, false);
  // the sample, then the table of its most frequent keys, then the rest of the column through the table
  hipError_t e = count_rounds(0, kHotSample, false);
  if (e == hipSuccess) e = launch_fill_u32(bin_n, kCountBins, 0u, s);
  if (e == hipSuccess) e = launch_fill_u32(reinterpret_cast<uint32_t *>(bin_sum), 2 * kCountBins, 0u, s);
  const int grid = (int)((n_keys + 255) / 256 < (int64_t)pl.blocks * 8 ? (n_keys + 255) / 256 : pl.blocks * 8);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(count_bins_kernel, dim3(grid), dim3(256), 0, s, counts, n_keys, bin_n, bin_sum);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(pick_hot_kernel, dim3(1), dim3(64), 0, s, bin_n, bin_sum, (uint64_t)kHotSample, tau, hot_n);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(collect_hot_kernel, dim3(grid), dim3(256), 0, s, counts, n_keys, tau, hot_keys, hot_n);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(hot_table_kernel, dim3(1), dim3(kHistThreads), 0, s, hot_keys, hot_n, table);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = count_rounds(kHotSample, n_fact, true);
  return e;
}

}  // namespace skew

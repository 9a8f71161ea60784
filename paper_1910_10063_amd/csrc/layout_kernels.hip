// Layout build kernels: key histogram, frequency rank sort, inversion,
// dimension copy and fact recoding (Section 3.1 and Section 3.2).
#include "device_common.h"
#include "kernels.h"
#include "query_common.h"

namespace skew {
namespace {

// ---------------------------------------------------------------------------
// Fill
// ---------------------------------------------------------------------------
__global__ void fill_u32_kernel(uint32_t *__restrict__ p, int64_t n, uint32_t v) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

// Index maintenance (Section 3.1): dimension rows [from, to) appended after
// the build become the least frequent items, Perm(i) = Rank(i) = i, with no
// occurrences counted; their columns go to the end of the permuted copy.
__global__ void append_rows_kernel(int32_t from, int32_t to, int32_t *__restrict__ perm, int32_t *__restrict__ rank,
                                   uint32_t *__restrict__ counts_by_rank, const int32_t *__restrict__ price,
                                   const int8_t *__restrict__ cat, int32_t *__restrict__ price_out,
                                   int8_t *__restrict__ cat_out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = from + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < to; i += stride) {
    perm[i] = (int32_t)i;
    rank[i] = (int32_t)i;
    if (counts_by_rank) counts_by_rank[i] = 0;
    if (price) price_out[i] = price[i];
    if (cat) cat_out[i] = cat[i];
  }
}

int grid_1d(int64_t n, int threads, int cap) {
  int64_t g = (n + threads - 1) / threads;
  if (g > cap) g = cap;
  return g < 1 ? 1 : (int)g;
}

// ---------------------------------------------------------------------------
// Key histogram.  The hot keys are not known before the layout exists, and
// even 1e5 keys of counters exceed LDS, so each workgroup privatises whatever
// keys it meets first in a small open-addressed LDS table (two probes); a key
// that finds no slot is counted with a global atomic.  Counts are exact in
// any interleaving.  Keys outside [0, n_keys) raise the error flag.
// ---------------------------------------------------------------------------
constexpr int kHistThreads = 1024;
constexpr int kHistSlotBits = 13;
constexpr int kHistSlots = 1 << kHistSlotBits;  // 8192 slots = 64 KB of LDS
constexpr int kHistUnroll = 2;

struct HistTable {
  int32_t *key;
  uint32_t *cnt;
};

__device__ __forceinline__ void hist_count(const HistTable &t, int32_t k, int32_t n_keys, uint32_t *counts,
                                           bool &bad) {
  if ((uint32_t)k >= (uint32_t)n_keys) {
    bad = true;
    return;
  }
  const uint32_t h = ((uint32_t)k * 0x9E3779B1u) >> (32 - kHistSlotBits);
#pragma unroll
  for (int probe = 0; probe < 2; ++probe) {
    const uint32_t s = (h + probe) & (kHistSlots - 1);
    int32_t cur = __hip_atomic_load(&t.key[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (cur == -1) {
      const int32_t old = atomicCAS(&t.key[s], -1, k);
      cur = (old == -1) ? k : old;
    }
    if (cur == k) {
      lds_add_u32(&t.cnt[s], 1u);
      return;
    }
  }
  global_add_u32(&counts[k], 1u);
}

__global__ __launch_bounds__(kHistThreads) void histogram_kernel(const int32_t *__restrict__ keys, int64_t n,
                                                                 int32_t n_keys, uint32_t *__restrict__ counts,
                                                                 int32_t *__restrict__ flag) {
  __shared__ int32_t slot_key[kHistSlots];
  __shared__ uint32_t slot_cnt[kHistSlots];
  for (int i = threadIdx.x; i < kHistSlots; i += blockDim.x) {
    slot_key[i] = -1;
    slot_cnt[i] = 0;
  }
  __syncthreads();
  const HistTable t{slot_key, slot_cnt};
  bool bad = false;

  const Split4 sp = split4(keys, n);
  const int64_t T = (int64_t)gridDim.x * blockDim.x;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid < sp.head) hist_count(t, keys[gid], n_keys, counts, bad);
  if (gid < n - sp.tail) hist_count(t, keys[sp.tail + gid], n_keys, counts, bad);
  const i32x4 *vk = reinterpret_cast<const i32x4 *>(keys + sp.head);
  int64_t v = gid;
  for (; v + (kHistUnroll - 1) * T < sp.nvec; v += kHistUnroll * T) {
    i32x4 x[kHistUnroll];
#pragma unroll
    for (int u = 0; u < kHistUnroll; ++u) x[u] = load_stream4(vk + v + u * T);
#pragma unroll
    for (int u = 0; u < kHistUnroll; ++u) {
      hist_count(t, x[u].x, n_keys, counts, bad);
      hist_count(t, x[u].y, n_keys, counts, bad);
      hist_count(t, x[u].z, n_keys, counts, bad);
      hist_count(t, x[u].w, n_keys, counts, bad);
    }
  }
  for (; v < sp.nvec; v += T) {
    const i32x4 x = load_stream4(vk + v);
    hist_count(t, x.x, n_keys, counts, bad);
    hist_count(t, x.y, n_keys, counts, bad);
    hist_count(t, x.z, n_keys, counts, bad);
    hist_count(t, x.w, n_keys, counts, bad);
  }
  if (bad) *flag = 1;
  __syncthreads();
  for (int i = threadIdx.x; i < kHistSlots; i += blockDim.x) {
    const int32_t k = slot_key[i];
    const uint32_t c = slot_cnt[i];
    if (k != -1 && c != 0) global_add_u32(&counts[k], c);
  }
}

// ---------------------------------------------------------------------------
// Rank sort: stable LSD radix sort of the key ids 0..n-1 by
// (maxv - count), 8-bit digits, which orders by decreasing count and keeps
// ascending key order among equal counts.  Tiles of 4096 elements; per pass
// an upsweep (digit histogram per tile), one scan over (digit, tile) and a
// downsweep that ranks every element among equal digits in index order.
// ---------------------------------------------------------------------------
constexpr int kSortThreads = 256;
constexpr int kSortRounds = kSortTile / kSortThreads;  // 16

// Lanes of this wave holding the same 8-bit digit (restricted to `active`).
__device__ __forceinline__ uint64_t match_digit(uint32_t d, uint64_t active) {
  uint64_t peers = active;
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t m = __ballot(bit);
    peers &= bit ? m : ~m;
  }
  return peers;
}

template <bool FIRST>
__device__ __forceinline__ uint32_t sort_key_at(const uint32_t *keys_in, int64_t i, uint32_t maxv) {
  return FIRST ? maxv - keys_in[i] : keys_in[i];
}

template <bool FIRST>
__global__ __launch_bounds__(kSortThreads) void radix_upsweep_kernel(const uint32_t *__restrict__ keys_in, int32_t n,
                                                                     int shift, uint32_t maxv,
                                                                     uint32_t *__restrict__ hist, int32_t tiles) {
  __shared__ uint32_t h[256];
  const int tid = threadIdx.x;
  h[tid] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  const uint64_t lt = (1ull << lane_id()) - 1ull;
  for (int r = 0; r < kSortRounds; ++r) {
    const int64_t i = base + (int64_t)r * kSortThreads + tid;
    const bool valid = i < n;
    const uint32_t d = valid ? (sort_key_at<FIRST>(keys_in, i, maxv) >> shift) & 255u : 0u;
    const uint64_t peers = match_digit(d, __ballot(valid));
    if (valid && (peers & lt) == 0) atomicAdd(&h[d], (uint32_t)__popcll(peers));
  }
  __syncthreads();
  hist[(int64_t)tid * tiles + blockIdx.x] = h[tid];
}

template <bool FIRST, bool LAST>
__global__ __launch_bounds__(kSortThreads) void radix_downsweep_kernel(
    const uint32_t *__restrict__ keys_in, const int32_t *__restrict__ vals_in, int32_t n, int shift, uint32_t maxv,
    const uint32_t *__restrict__ hist, int32_t tiles, uint32_t *__restrict__ keys_out, int32_t *__restrict__ vals_out) {
  __shared__ uint32_t run[256];        // next free position of each digit for this tile
  __shared__ uint32_t woff[4][256];    // per-wave digit counts, then per-wave start offsets
  const int tid = threadIdx.x;
  const int w = tid >> 6;
  const uint64_t lt = (1ull << lane_id()) - 1ull;
  run[tid] = hist[(int64_t)tid * tiles + blockIdx.x];
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  for (int r = 0; r < kSortRounds; ++r) {
    woff[0][tid] = 0;
    woff[1][tid] = 0;
    woff[2][tid] = 0;
    woff[3][tid] = 0;
    __syncthreads();
    const int64_t i = base + (int64_t)r * kSortThreads + tid;
    const bool valid = i < n;
    const uint32_t key = valid ? sort_key_at<FIRST>(keys_in, i, maxv) : 0u;
    const int32_t val = valid ? (FIRST ? (int32_t)i : vals_in[i]) : 0;
    const uint32_t d = (key >> shift) & 255u;
    const uint64_t peers = match_digit(d, __ballot(valid));
    const uint32_t rnk = (uint32_t)__popcll(peers & lt);
    if (valid && rnk == 0) woff[w][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    {
      const uint32_t c0 = woff[0][tid], c1 = woff[1][tid], c2 = woff[2][tid], c3 = woff[3][tid];
      const uint32_t b = run[tid];
      woff[0][tid] = b;
      woff[1][tid] = b + c0;
      woff[2][tid] = b + c0 + c1;
      woff[3][tid] = b + c0 + c1 + c2;
      run[tid] = b + c0 + c1 + c2 + c3;
    }
    __syncthreads();
    const uint32_t pos = woff[w][d] + rnk;
    if (valid && pos < (uint32_t)n) {
      if (LAST) {
        if (keys_out) keys_out[pos] = maxv - key;  // the count itself
      } else {
        keys_out[pos] = key;
      }
      vals_out[pos] = val;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Inverse, dimension copy, recode
// ---------------------------------------------------------------------------
__global__ void inverse_kernel(const int32_t *__restrict__ perm, int32_t n, int32_t *__restrict__ rank) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
    const int32_t k = perm[r];
    if ((uint32_t)k < (uint32_t)n) rank[k] = (int32_t)r;
  }
}

__global__ void permute_dims_kernel(const int32_t *__restrict__ perm, int32_t n, const int32_t *__restrict__ price,
                                    const int8_t *__restrict__ cat, int32_t *__restrict__ price_out,
                                    int8_t *__restrict__ cat_out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
    const int32_t k = perm[r];
    if ((uint32_t)k >= (uint32_t)n) continue;
    if (price) price_out[r] = price[k];
    if (cat) cat_out[r] = cat[k];
  }
}

constexpr int kRecodeThreads = 256;
constexpr int kRecodeUnroll = 4;

__device__ __forceinline__ int32_t recode_one(const int32_t *__restrict__ rank, int32_t n_keys, int32_t k) {
  return (uint32_t)k < (uint32_t)n_keys ? rank[k] : k;
}

__global__ __launch_bounds__(kRecodeThreads) void recode_kernel(const int32_t *keys, int64_t n,
                                                                const int32_t *__restrict__ rank, int32_t n_keys,
                                                                int32_t *out) {
  // keys may alias out (in-place recode): each element is read and written by one thread.
  const Split4 sp = split4(keys, n);
  const int64_t T = (int64_t)gridDim.x * blockDim.x;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid < sp.head) out[gid] = recode_one(rank, n_keys, keys[gid]);
  if (gid < n - sp.tail) out[sp.tail + gid] = recode_one(rank, n_keys, keys[sp.tail + gid]);
  const i32x4 *vk = reinterpret_cast<const i32x4 *>(keys + sp.head);
  i32x4 *vo = reinterpret_cast<i32x4 *>(out + sp.head);
  int64_t v = gid;
  for (; v + (kRecodeUnroll - 1) * T < sp.nvec; v += kRecodeUnroll * T) {
    i32x4 x[kRecodeUnroll];
#pragma unroll
    for (int u = 0; u < kRecodeUnroll; ++u) x[u] = load_stream4(vk + v + u * T);
#pragma unroll
    for (int u = 0; u < kRecodeUnroll; ++u) {
      i32x4 y;
      y.x = recode_one(rank, n_keys, x[u].x);
      y.y = recode_one(rank, n_keys, x[u].y);
      y.z = recode_one(rank, n_keys, x[u].z);
      y.w = recode_one(rank, n_keys, x[u].w);
      store_stream4(vo + v + u * T, y);
    }
  }
  for (; v < sp.nvec; v += T) {
    const i32x4 x = load_stream4(vk + v);
    i32x4 y;
    y.x = recode_one(rank, n_keys, x.x);
    y.y = recode_one(rank, n_keys, x.y);
    y.z = recode_one(rank, n_keys, x.z);
    y.w = recode_one(rank, n_keys, x.w);
    store_stream4(vo + v, y);
  }
}

// ---------------------------------------------------------------------------
// Recode with the hot keys in LDS.  Once the ranks are known, the hottest
// keys are known too (perm[0..T)): every workgroup inserts them, hottest
// first, into an LDS hash table of 4-slot buckets (a key whose bucket is full
// stays out), and each fact key is looked up there with one 16-byte LDS read
// before falling back to the rank array in global memory.  A slot is one
// word, (key >> 13) << 16 | rank, and the bucket is the low 13 bits of the
// key (8192 buckets x 4 slots = 128 KB), so the table serves key domains
// below 2^29 (larger domains gather every rank).
// ---------------------------------------------------------------------------
constexpr int kRecodeHotThreads = 1024;
constexpr int kRecodeTableWords = 32768;  // 128 KB of LDS
constexpr int kRecodeHotVecs = 4;

struct TagTable {
  static constexpr int kBucketBits = 13;
  static constexpr int kMaxKeys = 3 << kBucketBits;
  static constexpr uint32_t kEmpty = 0xFFFFFFFFu;  // rank 0xFFFF is never stored
  uint32_t *slots;  // [4 << kBucketBits]
  __device__ __forceinline__ TagTable(uint32_t *lds) : slots(lds) {}
  __device__ __forceinline__ static uint32_t bucket(uint32_t k) { return (k & ((1u << kBucketBits) - 1u)) * 4; }
  __device__ __forceinline__ void clear() {
    for (int i = threadIdx.x; i < (4 << kBucketBits); i += blockDim.x) slots[i] = kEmpty;
  }
  __device__ __forceinline__ void insert(int32_t k, int32_t r) {
    const uint32_t b = bucket((uint32_t)k);
    const uint32_t e = (((uint32_t)k >> kBucketBits) << 16) | (uint32_t)r;
    for (int j = 0; j < 4; ++j)
      if (atomicCAS(&slots[b + j], kEmpty, e) == kEmpty) break;
  }
  __device__ __forceinline__ bool find(uint32_t uk, int32_t *r) const {
    const uint32_t tag = uk >> kBucketBits;  // >= 2^16 for keys past 2^29: never equal to a stored tag
    const uint4 e = *reinterpret_cast<const uint4 *>(slots + bucket(uk));
    const bool h0 = e.x != kEmpty && (e.x >> 16) == tag, h1 = e.y != kEmpty && (e.y >> 16) == tag;
    const bool h2 = e.z != kEmpty && (e.z >> 16) == tag, h3 = e.w != kEmpty && (e.w >> 16) == tag;
    *r = (int32_t)((h0 ? e.x : (h1 ? e.y : (h2 ? e.z : e.w))) & 0xFFFFu);
    return h0 || h1 || h2 || h3;
  }
};

__device__ __forceinline__ int32_t recode_hot_one(const TagTable &tab, rsrc_t ranks, uint32_t n_keys, int32_t k) {
  const uint32_t uk = (uint32_t)k;
  int32_t rl;
  const bool hit = tab.find(uk, &rl);
  const int32_t rg = (int32_t)buffer_load_record(ranks, (int32_t)(hit ? 0xFFFFFFFFu : uk), 0, 0, 0);
  return uk < n_keys ? (hit ? rl : rg) : k;
}

__global__ __launch_bounds__(kRecodeHotThreads) void recode_hot_kernel(const int32_t *keys, int64_t n,
                                                                       const int32_t *__restrict__ rank,
                                                                       const int32_t *__restrict__ perm,
                                                                       int32_t n_keys, int32_t n_hot, int32_t *out) {
  __shared__ __align__(16) uint32_t lds[kRecodeTableWords];
  TagTable tab(lds);
  tab.clear();
  __syncthreads();
  for (int32_t r0 = 0; r0 < n_hot; r0 += kRecodeHotThreads) {  // hottest ranks claim slots first
    const int32_t r = r0 + (int32_t)threadIdx.x;
    if (r < n_hot) tab.insert(perm[r], r);
    __syncthreads();
  }
  const rsrc_t rk = record_buffer(rank, (uint32_t)n_keys);
  const uint32_t nk = (uint32_t)n_keys;
  // keys may alias out (in-place recode): each element is read and then written by one thread, and a
  // tile is loaded before the previous one is written, never after.
  const Split4 sp = split4(keys, n);
  if ((((uintptr_t)keys ^ (uintptr_t)out) & 15u) != 0) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride)
      out[j] = recode_hot_one(tab, rk, nk, keys[j]);
    return;
  }
  if (blockIdx.x == 0 && threadIdx.x < sp.head) out[threadIdx.x] = recode_hot_one(tab, rk, nk, keys[threadIdx.x]);
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x >= kWave && threadIdx.x - kWave < n - sp.tail) {
    const int64_t j = sp.tail + threadIdx.x - kWave;
    out[j] = recode_hot_one(tab, rk, nk, keys[j]);
  }
  const i32x4 *vk = reinterpret_cast<const i32x4 *>(keys + sp.head);
  i32x4 *vo = reinterpret_cast<i32x4 *>(out + sp.head);
  const int64_t per = (sp.nvec + gridDim.x - 1) / gridDim.x;
  const int64_t vb = (int64_t)blockIdx.x * per < sp.nvec ? (int64_t)blockIdx.x * per : sp.nvec;
  const int64_t ve = vb + per < sp.nvec ? vb + per : sp.nvec;
  constexpr int64_t kTile = (int64_t)kRecodeHotThreads * kRecodeHotVecs;
  const int64_t full_end = vb + ((ve - vb) / kTile) * kTile;
  auto resolve = [&](const i32x4(&x)[kRecodeHotVecs], int64_t base, bool guard) {
#pragma unroll
    for (int u = 0; u < kRecodeHotVecs; ++u) {
      const int64_t vi = base + u * kRecodeHotThreads + threadIdx.x;
      if (guard && vi >= ve) continue;
      i32x4 y;
      y.x = recode_hot_one(tab, rk, nk, x[u].x);
      y.y = recode_hot_one(tab, rk, nk, x[u].y);
      y.z = recode_hot_one(tab, rk, nk, x[u].z);
      y.w = recode_hot_one(tab, rk, nk, x[u].w);
      store_stream4(vo + vi, y);
    }
  };
  auto load_tile = [&](i32x4(&x)[kRecodeHotVecs], int64_t base) {
#pragma unroll
    for (int u = 0; u < kRecodeHotVecs; ++u) x[u] = load_stream4(vk + base + u * kRecodeHotThreads + threadIdx.x);
  };
  i32x4 xa[kRecodeHotVecs], xb[kRecodeHotVecs];
  int64_t base = vb;
  if (base < full_end) load_tile(xa, base);
  while (base < full_end) {
    int64_t nxt = base + kTile;
    load_tile(xb, nxt < full_end ? nxt : base);
    resolve(xa, base, false);
    base = nxt;
    if (base >= full_end) break;
    nxt = base + kTile;
    load_tile(xa, nxt < full_end ? nxt : base);
    resolve(xb, base, false);
    base = nxt;
  }
  if (full_end < ve) {
    i32x4 x[kRecodeHotVecs];
#pragma unroll
    for (int u = 0; u < kRecodeHotVecs; ++u) {
      const int64_t vi = full_end + u * kRecodeHotThreads + threadIdx.x;
      x[u] = vi < ve ? load_stream4(vk + vi) : i32x4{0, 0, 0, 0};
    }
    resolve(x, full_end, true);
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_1d(n, 256, 8192)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_histogram(const int32_t *keys, int64_t n, int32_t n_keys, uint32_t *counts, int32_t *flag,
                            const DeviceInfo &dev, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t need = (n + 4LL * kHistThreads - 1) / (4LL * kHistThreads);
  int grid = dev.cu_count * 2;
  if (need < grid) grid = (int)need;
  hipLaunchKernelGGL(histogram_kernel, dim3(grid), dim3(kHistThreads), 0, s, keys, n, n_keys, counts, flag);
  return hipGetLastError();
}

hipError_t launch_rank_sort(const uint32_t *counts_by_key, int32_t n_keys, int64_t n_fact, int32_t *perm,
                            uint32_t *counts_by_rank, uint32_t *keys_a, uint32_t *keys_b, int32_t *vals_a,
                            int32_t *vals_b, uint32_t *digit_hist, uint32_t *scan_scratch, hipStream_t s) {
  // Counts lie in [0, n_fact]; sort keys maxv - count need `bits` bits.
  int bits = 1;
  while (bits < 32 && ((uint64_t)1 << bits) <= (uint64_t)n_fact) ++bits;
  const uint32_t maxv = bits >= 32 ? 0xFFFFFFFFu : ((1u << bits) - 1u);
  const int passes = (bits + 7) / 8;
  const int32_t tiles = (int32_t)sort_tiles(n_keys);
  const int64_t total = 256LL * tiles;
  const uint32_t *kin = counts_by_key;
  const int32_t *vin = nullptr;
  for (int p = 0; p < passes; ++p) {
    const bool first = p == 0, last = p == passes - 1;
    const int shift = 8 * p;
    uint32_t *kout = last ? counts_by_rank : ((p & 1) ? keys_b : keys_a);
    int32_t *vout = last ? perm : ((p & 1) ? vals_b : vals_a);
    if (first)
      hipLaunchKernelGGL(radix_upsweep_kernel<true>, dim3(tiles), dim3(kSortThreads), 0, s, kin, n_keys, shift, maxv,
                         digit_hist, tiles);
    else
      hipLaunchKernelGGL(radix_upsweep_kernel<false>, dim3(tiles), dim3(kSortThreads), 0, s, kin, n_keys, shift, maxv,
                         digit_hist, tiles);
    hipError_t se = launch_exclusive_scan(digit_hist, total, nullptr, scan_scratch, s);
    if (se != hipSuccess) return se;
    if (first && last)
      hipLaunchKernelGGL((radix_downsweep_kernel<true, true>), dim3(tiles), dim3(kSortThreads), 0, s, kin, vin, n_keys,
                         shift, maxv, digit_hist, tiles, kout, vout);
    else if (first)
      hipLaunchKernelGGL((radix_downsweep_kernel<true, false>), dim3(tiles), dim3(kSortThreads), 0, s, kin, vin,
                         n_keys, shift, maxv, digit_hist, tiles, kout, vout);
    else if (last)
      hipLaunchKernelGGL((radix_downsweep_kernel<false, true>), dim3(tiles), dim3(kSortThreads), 0, s, kin, vin,
                         n_keys, shift, maxv, digit_hist, tiles, kout, vout);
    else
      hipLaunchKernelGGL((radix_downsweep_kernel<false, false>), dim3(tiles), dim3(kSortThreads), 0, s, kin, vin,
                         n_keys, shift, maxv, digit_hist, tiles, kout, vout);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    kin = kout;
    vin = vout;
  }
  return hipSuccess;
}

hipError_t launch_inverse(const int32_t *perm, int32_t n, int32_t *rank, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(inverse_kernel, dim3(grid_1d(n, 256, 16384)), dim3(256), 0, s, perm, n, rank);
  return hipGetLastError();
}

hipError_t launch_append_rows(int32_t from, int32_t to, int32_t *perm, int32_t *rank, uint32_t *counts_by_rank,
                              const int32_t *price, const int8_t *cat, int32_t *price_out, int8_t *cat_out,
                              hipStream_t s) {
  if (to <= from) return hipSuccess;
  hipLaunchKernelGGL(append_rows_kernel, dim3(grid_1d(to - from, 256, 16384)), dim3(256), 0, s, from, to, perm, rank,
                     counts_by_rank, price, cat, price_out, cat_out);
  return hipGetLastError();
}

hipError_t launch_permute_dims(const int32_t *perm, int32_t n, const int32_t *price, const int8_t *cat,
                               int32_t *price_out, int8_t *cat_out, hipStream_t s) {
  if (n <= 0 || (!price && !cat)) return hipSuccess;
  hipLaunchKernelGGL(permute_dims_kernel, dim3(grid_1d(n, 256, 16384)), dim3(256), 0, s, perm, n, price, cat,
                     price_out, cat_out);
  return hipGetLastError();
}

hipError_t launch_recode(const int32_t *keys, int64_t n, const int32_t *rank, const int32_t *perm, int32_t n_keys,
                         int32_t *out, const DeviceInfo &dev, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (perm && n >= (int64_t)dev.cu_count * 65536 && n_keys <= (1 << 29)) {  // large columns: hot keys in LDS
    const int32_t n_hot = n_keys < TagTable::kMaxKeys ? n_keys : TagTable::kMaxKeys;
    hipLaunchKernelGGL(recode_hot_kernel, dim3(dev.cu_count), dim3(kRecodeHotThreads), 0, s, keys, n, rank,
                       perm, n_keys, n_hot, out);
    return hipGetLastError();
  }
  const int64_t need = (n + 4LL * kRecodeThreads - 1) / (4LL * kRecodeThreads);
  int grid = dev.cu_count * 8;
  if (need < grid) grid = (int)need;
  hipLaunchKernelGGL(recode_kernel, dim3(grid), dim3(kRecodeThreads), 0, s, keys, n, rank, n_keys, out);
  return hipGetLastError();
}

}  // namespace skew

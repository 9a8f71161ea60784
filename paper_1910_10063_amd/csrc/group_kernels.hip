// Grouped SUM/COUNT (Q3 of Section 1): hot groups privatised per workgroup in
// LDS with per-lane copies of the hottest ones (Section 4.2.2, Section 4.3).
// Cold groups either go to shared global atomics (single pass) or are written
// to a cold buffer, partitioned by group slice and aggregated from LDS bins
// of each slice in a second pass (the threshold split of Section 4.2.1).
#include "kernels.h"
#include "profiler.h"
#include "query_common.h"

namespace skew {
namespace {

__global__ void group_prep_kernel(uint64_t *__restrict__ acc_sum, uint64_t *__restrict__ acc_cnt, int32_t m,
                                  int32_t *flag) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid == 0) *flag = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = gid; i < m; i += stride) {
    acc_sum[i] = 0;
    acc_cnt[i] = 0;
  }
}

constexpr int kGroupUnroll = 2;
constexpr int kHashSlotBits = 13;
constexpr int kHashSlots = 1 << kHashSlotBits;  // 8192 slots x 16 B = 128 KB

struct GroupCtx {
  int32_t m;
  int32_t t;      // groups [0, t) live in LDS
  int32_t ncopy;  // groups [0, ncopy) have per-lane copies, ncopy = min(t, kGroupCopies)
  uint64_t *acc_sum;
  uint64_t *acc_cnt;
  bool bad;
  // range mode: one LDS array per accumulator, the per-lane copies of groups
  // [0, ncopy) at [g * 64 + lane] followed by the bins of groups [0, t) at
  // [kCopySlots + g]; one array keeps every update a single LDS atomic.
  uint64_t *hot_sum;
  uint32_t *hot_cnt;
  uint64_t *pack;      // pass 1 of the partitioned form: packed bins, same slot order
  int32_t *slot_key;   // hash mode [kHashSlots]
  uint64_t *slot_sum;
  uint32_t *slot_cnt;
};

__device__ __forceinline__ void group_global(const GroupCtx &c, int32_t g, int32_t v) {
  global_add_u64(&c.acc_sum[g], (uint64_t)(int64_t)v);
  global_add_u64(&c.acc_cnt[g], 1ull);
}

constexpr int kCopySlots = kGroupCopies * kWave;

// A hot group (g < t): its per-lane copy (the hottest groups, never contended
// within a wave) or its workgroup bin.
__device__ __forceinline__ void group_hot(const GroupCtx &c, int32_t g, int32_t v) {
  const int i = g < c.ncopy ? g * kWave + lane_id() : kCopySlots + g;
  lds_add_u64(&c.hot_sum[i], (uint64_t)(int64_t)v);
  lds_add_u32(&c.hot_cnt[i], 1u);
}

template <int MODE>
__device__ __forceinline__ void group_one(GroupCtx &c, int32_t g, int32_t v) {
  if ((uint32_t)g >= (uint32_t)c.m) {
    c.bad = true;
    return;
  }
  if (MODE == kGroupRange) {
    if (g < c.t) group_hot(c, g, v);
    else group_global(c, g, v);
  } else if (MODE == kGroupHash) {
    const uint32_t h = ((uint32_t)g * 0x9E3779B1u) >> (32 - kHashSlotBits);
#pragma unroll
    for (int probe = 0; probe < 2; ++probe) {
      const uint32_t s = (h + probe) & (kHashSlots - 1);
      int32_t cur = __hip_atomic_load(&c.slot_key[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      if (cur == -1) {
        const int32_t old = atomicCAS(&c.slot_key[s], -1, g);
        cur = (old == -1) ? g : old;
      }
      if (cur == g) {
        lds_add_u64(&c.slot_sum[s], (uint64_t)(int64_t)v);
        lds_add_u32(&c.slot_cnt[s], 1u);
        return;
      }
    }
    group_global(c, g, v);
  } else {
    group_global(c, g, v);
  }
}

// LDS layout of the single pass's range mode: hot_sum[kCopySlots + t] |
// hot_cnt[kCopySlots + t].
__device__ __forceinline__ void group_range_init(GroupCtx &c, unsigned char *smem, int32_t t) {
  c.hot_sum = reinterpret_cast<uint64_t *>(smem);
  c.hot_cnt = reinterpret_cast<uint32_t *>(c.hot_sum + kCopySlots + t);
  for (int i = threadIdx.x; i < kCopySlots + t; i += blockDim.x) {
    c.hot_sum[i] = 0;
    c.hot_cnt[i] = 0;
  }
}

// Flush the range-mode LDS bins into the shared accumulators.
__device__ __forceinline__ void group_range_flush(const GroupCtx &c) {
  const int w = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  for (int g = w; g < c.ncopy; g += nw) {
    const uint64_t s = wave_sum_u64(c.hot_sum[g * kWave + lane_id()]);
    const uint64_t k = wave_sum_u64((uint64_t)c.hot_cnt[g * kWave + lane_id()]);
    if (lane_id() == 0 && k) {
      global_add_u64(&c.acc_sum[g], s);
      global_add_u64(&c.acc_cnt[g], k);
    }
  }
  for (int g = c.ncopy + threadIdx.x; g < c.t; g += blockDim.x) {
    const uint32_t k = c.hot_cnt[kCopySlots + g];
    if (k) {
      global_add_u64(&c.acc_sum[g], c.hot_sum[kCopySlots + g]);
      global_add_u64(&c.acc_cnt[g], (uint64_t)k);
    }
  }
}

// ---------------------------------------------------------------------------
// Single pass.
// ---------------------------------------------------------------------------
template <int MODE>
__global__ __launch_bounds__(kGroupThreads) void group_kernel(const int32_t *__restrict__ keys,
                                                              const int32_t *__restrict__ vals, int64_t n, int32_t m,
                                                              int32_t t, uint64_t *__restrict__ acc_sum,
                                                              uint64_t *__restrict__ acc_cnt, int32_t *flag) {
  extern __shared__ __align__(16) unsigned char smem[];
  GroupCtx c;
  c.m = m;
  c.t = t;
  c.ncopy = t < kGroupCopies ? t : kGroupCopies;
  c.acc_sum = acc_sum;
  c.acc_cnt = acc_cnt;
  c.bad = false;
  if (MODE == kGroupRange) {
    group_range_init(c, smem, t);
  } else if (MODE == kGroupHash) {
    c.slot_sum = reinterpret_cast<uint64_t *>(smem);
    c.slot_key = reinterpret_cast<int32_t *>(c.slot_sum + kHashSlots);
    c.slot_cnt = reinterpret_cast<uint32_t *>(c.slot_key + kHashSlots);
    for (int i = threadIdx.x; i < kHashSlots; i += blockDim.x) {
      c.slot_sum[i] = 0;
      c.slot_key[i] = -1;
      c.slot_cnt[i] = 0;
    }
  }
  __syncthreads();

  // keys and values share the row index; they are aligned together only when
  // their addresses agree mod 16, otherwise the scalar loop takes all rows.
  const bool vec_ok = (((uintptr_t)keys ^ (uintptr_t)vals) & 15u) == 0;
  const int64_t T = (int64_t)gridDim.x * blockDim.x;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (vec_ok) {
    const Split4 sp = split4(keys, n);
    if (gid < sp.head) group_one<MODE>(c, keys[gid], vals[gid]);
    if (gid < n - sp.tail) group_one<MODE>(c, keys[sp.tail + gid], vals[sp.tail + gid]);
    const i32x4 *vk = reinterpret_cast<const i32x4 *>(keys + sp.head);
    const i32x4 *vv = reinterpret_cast<const i32x4 *>(vals + sp.head);
    int64_t v = gid;
    for (; v + (kGroupUnroll - 1) * T < sp.nvec; v += kGroupUnroll * T) {
      i32x4 x[kGroupUnroll], y[kGroupUnroll];
#pragma unroll
      for (int u = 0; u < kGroupUnroll; ++u) {
        x[u] = load_stream4(vk + v + u * T);
        y[u] = load_stream4(vv + v + u * T);
      }
#pragma unroll
      for (int u = 0; u < kGroupUnroll; ++u) {
        group_one<MODE>(c, x[u].x, y[u].x);
        group_one<MODE>(c, x[u].y, y[u].y);
        group_one<MODE>(c, x[u].z, y[u].z);
        group_one<MODE>(c, x[u].w, y[u].w);
      }
    }
    for (; v < sp.nvec; v += T) {
      const i32x4 x = load_stream4(vk + v);
      const i32x4 y = load_stream4(vv + v);
      group_one<MODE>(c, x.x, y.x);
      group_one<MODE>(c, x.y, y.y);
      group_one<MODE>(c, x.z, y.z);
      group_one<MODE>(c, x.w, y.w);
    }
  } else {
    for (int64_t i = gid; i < n; i += T) group_one<MODE>(c, load_stream1(keys + i), load_stream1(vals + i));
  }
  if (c.bad) *flag = 1;
  __syncthreads();

  if (MODE == kGroupRange) {
    group_range_flush(c);
  } else if (MODE == kGroupHash) {
    for (int s = threadIdx.x; s < kHashSlots; s += blockDim.x) {
      const int32_t g = c.slot_key[s];
      const uint32_t k = c.slot_cnt[s];
      if (g != -1 && k) {
        global_add_u64(&acc_sum[g], c.slot_sum[s]);
        global_add_u64(&acc_cnt[g], (uint64_t)k);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Partitioned form, pass 1: rows of hot groups into LDS bins; every other
// valid row appended to this workgroup's segment of the cold buffer of its
// stream (4-byte records or pairs, below) and counted in its slice
// (g >> wshift; slices cover all groups, so that a hot row the bins cannot
// take is resolved like a cold one).
//
// A bin is one 64-bit word, count << 40 | sum, updated by a single LDS atomic.
// It takes rows whose value lies in [0, 2^16); it stays exact while it sees
// fewer than 2^24 rows, since the sum then stays below 2^40, and the plan
// gives every workgroup fewer than 2^24 rows per launch.  Rows of hot groups
// with other values go to the cold buffer.
// ---------------------------------------------------------------------------
constexpr int kSplitVecs = 2;  // 16-byte vectors of keys (and of values) per lane per batch
constexpr int kPackShift = 40;
constexpr uint64_t kPackSumMask = (1ull << kPackShift) - 1ull;
constexpr uint32_t kPackValueLimit = 1u << 16;
constexpr int64_t kPackMaxRows = 1LL << 24;  // rows a workgroup may give one launch of pass 1

// LDS layout of pass 1: pack[kCopySlots + t + kWave] (per-lane copies, bins,
// one sink slot per lane that is never flushed).
__device__ __forceinline__ void group_pack_init(GroupCtx &c, unsigned char *smem) {
  c.pack = reinterpret_cast<uint64_t *>(smem);
  for (int i = threadIdx.x; i < kCopySlots + c.t + kWave; i += blockDim.x) c.pack[i] = 0;
}

// Hot update without branches: lanes whose row is not taken add into a sink
// slot of their own (kCopySlots + t + lane).
__device__ __forceinline__ void group_pack_or_sink(const GroupCtx &c, bool h, uint32_t g, int32_t v, uint32_t sink) {
  const uint32_t i = h ? (g < (uint32_t)c.ncopy ? g * kWave + lane_id() : kCopySlots + g) : sink;
  lds_add_u64(&c.pack[i], (1ull << kPackShift) | (uint32_t)v);
}

__device__ __forceinline__ void group_pack_flush(const GroupCtx &c) {
  const int w = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  for (int g = w; g < c.ncopy; g += nw) {
    const uint64_t x = c.pack[g * kWave + lane_id()];
    const uint64_t s = wave_sum_u64(x & kPackSumMask);
    const uint64_t k = wave_sum_u64(x >> kPackShift);
    if (lane_id() == 0 && k) {
      global_add_u64(&c.acc_sum[g], s);
      global_add_u64(&c.acc_cnt[g], k);
    }
  }
  for (int g = c.ncopy + threadIdx.x; g < c.t; g += blockDim.x) {
    const uint64_t x = c.pack[kCopySlots + g];
    if (x) {
      global_add_u64(&c.acc_sum[g], x & kPackSumMask);
      global_add_u64(&c.acc_cnt[g], x >> kPackShift);
    }
  }
}

struct PairSeg {  // this workgroup's segment; stores a chunk of (group, value) pairs
  rsrc_t keys, vals;
  __device__ __forceinline__ void operator()(const uint32_t (&col)[2], int32_t idx, bool ok) const {
    const int32_t i = ok ? idx : -1;  // -1: out of range, dropped
    buffer_store_record((int32_t)col[0], keys, i, 0, 0, 0);
    buffer_store_record((int32_t)col[1], vals, i, 0, 0, 0);
  }
};

// Narrow cold rows: over at most 2^20 groups, a cold row whose value lies in
// [0, 2^12) travels as one 4-byte record, group << 12 | value, in a stream
// of its own (segments, slice counts, scatter and pass 3), at half the bytes
// of a (group, value) pair.  The other cold rows take the pair stream.  Both
// streams share one slice table: rows [0, np) of the slice counts are the
// narrow slices (np = P, or 0 when the groups do not fit), rows [np, np + P)
// the pair slices, so one plan places both.
constexpr int kNarrowShift = kGroupNarrowShift;
constexpr uint32_t kNarrowValueLimit = 1u << kNarrowShift;
constexpr int64_t kNarrowMaxGroups = 1LL << (32 - kNarrowShift);

struct NarrowSeg {  // this workgroup's narrow segment
  rsrc_t recs;
  __device__ __forceinline__ void operator()(const uint32_t (&col)[1], int32_t idx, bool ok) const {
    buffer_store_record((int32_t)col[0], recs, ok ? idx : -1, 0, 0, 0);
  }
};

struct ColdOut {
  ColdSink pair, narrow;  // shared slice counts, one item counter each
  WaveChunk<2> cp;
  WaveChunk<1> cn;
  PairSeg seg;
  NarrowSeg segn;
  uint32_t np;  // narrow slices; 0: every cold row is a pair
};

// Cold rows to their stream: one chunk append per stream (a stream with no
// row in the slot costs one ballot) and one count in the shared table.
template <int N>
__device__ __forceinline__ void cold_append_two(ColdOut &co, const uint32_t (&g)[N], const int32_t (&v)[N],
                                                const bool (&cold)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const bool nw = cold[i] && co.np != 0u && (uint32_t)v[i] < kNarrowValueLimit;
    const bool pr = cold[i] && !nw;
    if (co.np != 0u) {  // uniform
      const uint32_t rec[1] = {(g[i] << kNarrowShift) | (uint32_t)v[i]};
      chunk_append(co.narrow, co.cn, nw, rec, co.segn);
    }
    const uint32_t pair[2] = {g[i], (uint32_t)v[i]};
    chunk_append(co.pair, co.cp, pr, pair, co.seg);
    lds_add_u32(&co.pair.hist[cold[i] ? (g[i] >> co.pair.wshift) + (nw ? 0u : co.np) : co.pair.sink], 1u);
  }
}

template <int V>
__device__ __forceinline__ void group_split_batch(GroupCtx &c, ColdOut &co, uint32_t hot_sink, const i32x4 (&x)[V],
                                                  const i32x4 (&y)[V], const bool (&valid)[V]) {
  uint32_t g[4 * V];
  int32_t v[4 * V];
  bool cold[4 * V];
#pragma unroll
  for (int u = 0; u < V; ++u) {
    g[4 * u] = (uint32_t)x[u].x, g[4 * u + 1] = (uint32_t)x[u].y;
    g[4 * u + 2] = (uint32_t)x[u].z, g[4 * u + 3] = (uint32_t)x[u].w;
    v[4 * u] = y[u].x, v[4 * u + 1] = y[u].y, v[4 * u + 2] = y[u].z, v[4 * u + 3] = y[u].w;
  }
#pragma unroll
  for (int i = 0; i < 4 * V; ++i) {
    const bool ok = valid[i / 4];
    const bool in = ok && g[i] < (uint32_t)c.m;
    c.bad |= ok && !in;
    const bool h = in && g[i] < (uint32_t)c.t && (uint32_t)v[i] < kPackValueLimit;
    cold[i] = in && !h;
    group_pack_or_sink(c, h, g[i], v[i], hot_sink);
  }
  cold_append_two(co, g, v, cold);
}

__device__ __forceinline__ void group_split_one(GroupCtx &c, ColdOut &co, uint32_t hot_sink, bool valid, int32_t gi,
                                                int32_t vi) {
  const uint32_t g[1] = {(uint32_t)gi};
  const int32_t v[1] = {vi};
  const bool in = valid && g[0] < (uint32_t)c.m;
  c.bad |= valid && !in;
  const bool h = in && g[0] < (uint32_t)c.t && (uint32_t)vi < kPackValueLimit;
  const bool cold[1] = {in && !h};
  group_pack_or_sink(c, h, g[0], vi, hot_sink);
  cold_append_two(co, g, v, cold);
}

__global__ __launch_bounds__(kGroupThreads) void group_split_kernel(
    const int32_t *__restrict__ keys, const int32_t *__restrict__ vals, int64_t n, int32_t m, int32_t t, int32_t P,
    int32_t wshift, int32_t np, uint64_t *__restrict__ acc_sum, uint64_t *__restrict__ acc_cnt, int32_t *flag,
    int32_t *__restrict__ seg_keys, int32_t *__restrict__ seg_vals, int32_t *__restrict__ seg_recs, int64_t seg_cap,
    uint32_t *__restrict__ seg_count, uint32_t *__restrict__ seg_count_n, uint32_t *__restrict__ hist) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int32_t Q = np + P;  // rows of the slice table: narrow slices, then pair slices
  GroupCtx c;
  c.m = m;
  c.t = t;
  c.ncopy = t < kGroupCopies ? t : kGroupCopies;
  c.acc_sum = acc_sum;
  c.acc_cnt = acc_cnt;
  c.bad = false;
  group_pack_init(c, smem);
  uint32_t *lhist = reinterpret_cast<uint32_t *>(c.pack + kCopySlots + t + kWave);
  uint32_t *lcount = lhist + Q + kWave;  // [0]: pair items, [1]: narrow items
  for (int p = threadIdx.x; p < Q + kWave; p += blockDim.x) lhist[p] = 0;
  if (threadIdx.x < 2) lcount[threadIdx.x] = 0;
  __syncthreads();
  ColdOut co;
  co.pair.count = lcount;
  co.pair.hist = lhist;
  co.pair.t = 0;  // slices of all groups
  co.pair.wshift = wshift;
  co.pair.sink = (uint32_t)Q + lane_id();
  co.narrow = co.pair;
  co.narrow.count = lcount + 1;
  co.np = (uint32_t)np;
  co.seg.keys = record_buffer(seg_keys + (int64_t)blockIdx.x * seg_cap, (uint32_t)seg_cap);
  co.seg.vals = record_buffer(seg_vals + (int64_t)blockIdx.x * seg_cap, (uint32_t)seg_cap);
  co.segn.recs = record_buffer(seg_recs + (int64_t)blockIdx.x * seg_cap, np ? (uint32_t)seg_cap : 0u);
  const uint32_t hot_sink = (uint32_t)(kCopySlots + t) + lane_id();
  co.cp.n = 0;
  co.cp.col[0] = co.cp.col[1] = 0;
  co.cn.n = 0;
  co.cn.col[0] = 0;

  // Workgroup b owns rows [b * per, (b + 1) * per) (in 4-row vectors when the
  // two columns are aligned together, else in single rows).
  const bool vec_ok = (((uintptr_t)keys ^ (uintptr_t)vals) & 15u) == 0;
  if (vec_ok) {
    const Split4 sp = split4(keys, n);
    {  // scalar head (block 0, lanes 0-2) and tail (last block, lanes 64-66)
      int64_t i = -1;
      if (blockIdx.x == 0 && threadIdx.x < sp.head) i = threadIdx.x;
      if (blockIdx.x == gridDim.x - 1 && threadIdx.x >= 64 && threadIdx.x - 64 < n - sp.tail)
        i = sp.tail + threadIdx.x - 64;
      group_split_one(c, co, hot_sink, i >= 0, i >= 0 ? keys[i] : 0, i >= 0 ? vals[i] : 0);
    }
    const int64_t per = (sp.nvec + gridDim.x - 1) / gridDim.x;
    const int64_t vb = (int64_t)blockIdx.x * per < sp.nvec ? (int64_t)blockIdx.x * per : sp.nvec;
    const int64_t ve = vb + per < sp.nvec ? vb + per : sp.nvec;
    const i32x4 *vk = reinterpret_cast<const i32x4 *>(keys + sp.head);
    const i32x4 *vv = reinterpret_cast<const i32x4 *>(vals + sp.head);
    const int64_t tile_vecs = (int64_t)kGroupThreads * kSplitVecs;
    const int64_t full_end = vb + ((ve - vb) / tile_vecs) * tile_vecs;
    bool all_valid[kSplitVecs];
#pragma unroll
    for (int u = 0; u < kSplitVecs; ++u) all_valid[u] = true;
    auto load_tile = [&](i32x4(&x)[kSplitVecs], i32x4(&y)[kSplitVecs], int64_t base) {
#pragma unroll
      for (int u = 0; u < kSplitVecs; ++u) {
        x[u] = load_stream4(vk + base + u * kGroupThreads + threadIdx.x);
        y[u] = load_stream4(vv + base + u * kGroupThreads + threadIdx.x);
      }
    };
    i32x4 xa[kSplitVecs], ya[kSplitVecs], xb[kSplitVecs], yb[kSplitVecs];
    int64_t base = vb;
    if (base < full_end) load_tile(xa, ya, base);
    while (base < full_end) {  // the next tile is loaded while the current one is processed
      int64_t nxt = base + tile_vecs;
      load_tile(xb, yb, nxt < full_end ? nxt : base);
      group_split_batch<kSplitVecs>(c, co, hot_sink, xa, ya, all_valid);
      base = nxt;
      if (base >= full_end) break;
      nxt = base + tile_vecs;
      load_tile(xa, ya, nxt < full_end ? nxt : base);
      group_split_batch<kSplitVecs>(c, co, hot_sink, xb, yb, all_valid);
      base = nxt;
    }
    if (full_end < ve) {  // last partial tile
      i32x4 x[kSplitVecs], y[kSplitVecs];
      bool valid[kSplitVecs];
#pragma unroll
      for (int u = 0; u < kSplitVecs; ++u) {
        const int64_t vi = full_end + u * kGroupThreads + threadIdx.x;
        valid[u] = vi < ve;
        x[u] = valid[u] ? load_stream4(vk + vi) : i32x4{0, 0, 0, 0};
        y[u] = valid[u] ? load_stream4(vv + vi) : i32x4{0, 0, 0, 0};
      }
      group_split_batch<kSplitVecs>(c, co, hot_sink, x, y, valid);
    }
  } else {
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t rb = (int64_t)blockIdx.x * per < n ? (int64_t)blockIdx.x * per : n;
    const int64_t re = rb + per < n ? rb + per : n;
    for (int64_t base = rb; base < re; base += blockDim.x) {
      const int64_t i = base + threadIdx.x;
      const bool valid = i < re;
      group_split_one(c, co, hot_sink, valid, valid ? load_stream1(keys + i) : 0,
                      valid ? load_stream1(vals + i) : 0);
    }
  }
  chunk_drain(co.pair, co.cp, co.seg);
  if (np) chunk_drain(co.narrow, co.cn, co.segn);
  if (c.bad) *flag = 1;
  __syncthreads();
  if (threadIdx.x == 0) seg_count[blockIdx.x] = lcount[0] < seg_cap ? lcount[0] : (uint32_t)seg_cap;
  if (threadIdx.x == 1) seg_count_n[blockIdx.x] = lcount[1] < seg_cap ? lcount[1] : (uint32_t)seg_cap;
  for (int p = threadIdx.x; p < Q; p += blockDim.x) hist[(int64_t)p * gridDim.x + blockIdx.x] = lhist[p];
  group_pack_flush(c);
}

// ---------------------------------------------------------------------------
// Partitioned form, pass 3, one launch per stream: the slice-ordered items
// (pairs: 2-byte group offsets inside their slice and 4-byte values; narrow:
// one word, offset << 12 | value) are cut into one contiguous share per
// workgroup, balanced over items plus the cost of flushing each slice; the
// workgroup sums the items of each slice its share touches in LDS bins (W
// groups) and flushes the bins into the shared accumulators before it moves
// to the next slice.  slice_off[0..P] are positions in the item arrays (the
// pair stream's start after the narrow items).
// ---------------------------------------------------------------------------
constexpr int kSliceVecs = 2;  // 8-pair vectors per lane per batch

struct PairVec {
  i32x4 l;       // 8 group offsets, 2 bytes each
  i32x4 v0, v1;  // their 8 values
};

__device__ __forceinline__ void slice_flush(uint64_t *bsum, uint32_t *bcnt, int32_t slen, int64_t sbase,
                                            uint64_t *acc_sum, uint64_t *acc_cnt) {
  for (int i = threadIdx.x; i < slen; i += blockDim.x) {
    const uint32_t k = bcnt[i];
    if (k) {
      global_add_u64(&acc_sum[sbase + i], bsum[i]);
      global_add_u64(&acc_cnt[sbase + i], (uint64_t)k);
      bsum[i] = 0;
      bcnt[i] = 0;
    }
  }
}

template <bool NARROW>
__global__ __launch_bounds__(kGroupThreads) void group_slice_kernel(
    const uint16_t *__restrict__ locals, const int32_t *__restrict__ vals, const uint32_t *__restrict__ slice_off,
    int32_t P, int32_t m, int32_t t, int32_t wshift, uint64_t *__restrict__ acc_sum, uint64_t *__restrict__ acc_cnt) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int32_t W = 1 << wshift;
  uint64_t *bsum = reinterpret_cast<uint64_t *>(smem);
  uint32_t *bcnt = reinterpret_cast<uint32_t *>(bsum + W);
  uint32_t *soff = bcnt + W;
  for (int i = threadIdx.x; i < W; i += blockDim.x) {
    bsum[i] = 0;
    bcnt[i] = 0;
  }
  const uint32_t first = slice_off[0];  // items of this stream are [first, slice_off[P])
  for (int p = threadIdx.x; p <= P; p += blockDim.x) soff[p] = slice_off[p] - first;
  __syncthreads();
  uint32_t lo, hi;
  balanced_share(soff, P, 2u * (uint32_t)W, blockIdx.x, gridDim.x, &lo, &hi);
  int32_t p = lo < hi ? slice_of_item(soff, P, lo) : P;
  lo += first;  // back to positions in the item arrays (16-byte aligned at position 0)
  hi += first;
  const i32x4 *vl = reinterpret_cast<const i32x4 *>(locals);
  const i32x4 *vv = reinterpret_cast<const i32x4 *>(vals);
  auto add = [&](uint32_t local, int32_t v) {  // local < W by construction
    lds_add_u64(&bsum[local], (uint64_t)(int64_t)v);
    lds_add_u32(&bcnt[local], 1u);
  };
  auto add_rec = [&](uint32_t r) { add(r >> kNarrowShift, (int32_t)(r & (kNarrowValueLimit - 1u))); };
  for (uint32_t at = lo; at < hi; ++p) {
    const uint32_t end = soff[p + 1] + first < hi ? soff[p + 1] + first : hi;
    if (end <= at) continue;
    const int64_t sbase = (int64_t)t + ((int64_t)p << wshift);
    const int32_t slen = (int32_t)((int64_t)m - sbase < W ? (int64_t)m - sbase : W);
    if (NARROW) {
      walk_items<4, 2 * kSliceVecs, kGroupThreads, i32x4>(
          at, end, [&](uint32_t i) { add_rec((uint32_t)vals[i]); }, [&](uint32_t vi) { return load_stream4(vv + vi); },
          [&](const i32x4(&x)[2 * kSliceVecs], const bool(&valid)[2 * kSliceVecs]) {
#pragma unroll
            for (int u = 0; u < 2 * kSliceVecs; ++u) {
              if (!valid[u]) continue;
              add_rec((uint32_t)x[u].x);
              add_rec((uint32_t)x[u].y);
              add_rec((uint32_t)x[u].z);
              add_rec((uint32_t)x[u].w);
            }
          });
    } else {
    walk_items<8, kSliceVecs, kGroupThreads, PairVec>(
        at, end, [&](uint32_t i) { add(locals[i], vals[i]); },
        [&](uint32_t vi) { return PairVec{load_stream4(vl + vi), load_stream4(vv + 2 * vi), load_stream4(vv + 2 * vi + 1)}; },
        [&](const PairVec(&x)[kSliceVecs], const bool(&valid)[kSliceVecs]) {
#pragma unroll
          for (int u = 0; u < kSliceVecs; ++u) {
            if (!valid[u]) continue;
            const uint32_t d[4] = {(uint32_t)x[u].l.x, (uint32_t)x[u].l.y, (uint32_t)x[u].l.z, (uint32_t)x[u].l.w};
            const int32_t v[8] = {x[u].v0.x, x[u].v0.y, x[u].v0.z, x[u].v0.w,
                                  x[u].v1.x, x[u].v1.y, x[u].v1.z, x[u].v1.w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              add(d[j] & 0xFFFFu, v[2 * j]);
              add(d[j] >> 16, v[2 * j + 1]);
            }
          }
        });
    }
    __syncthreads();
    slice_flush(bsum, bcnt, slen, sbase, acc_sum, acc_cnt);
    __syncthreads();
    at = end;
  }
}

__global__ void unpermute_kernel(const uint64_t *__restrict__ acc_sum, const uint64_t *__restrict__ acc_cnt,
                                 const int32_t *__restrict__ perm, int32_t m, int64_t *__restrict__ out_sum,
                                 int64_t *__restrict__ out_cnt) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < m; r += stride) {
    const int32_t k = perm[r];
    if ((uint32_t)k >= (uint32_t)m) continue;  // perm must be a permutation of [0, m)
    out_sum[k] = (int64_t)acc_sum[r];
    out_cnt[k] = (int64_t)acc_cnt[r];
  }
}

int grid_1d(int64_t n, int threads, int cap) {
  int64_t g = (n + threads - 1) / threads;
  if (g > cap) g = cap;
  return g < 1 ? 1 : (int)g;
}

template <typename K>
void allow_lds(K kernel, size_t bytes) {
  if (bytes > 48 * 1024)
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)bytes);
}

}  // namespace

// ---------------------------------------------------------------------------
// Capacities and launchers
// ---------------------------------------------------------------------------
size_t group_lds_bytes(int32_t hot_groups) {
  return (size_t)kGroupCopies * kWave * 12 + (size_t)(hot_groups > 0 ? hot_groups : 0) * 12;
}

int32_t group_max_hot_groups(const DeviceInfo &dev) {
  const size_t fixed = group_lds_bytes(0);
  if (dev.lds_per_block <= fixed) return 0;
  return (int32_t)((dev.lds_per_block - fixed) / 12);
}

size_t group_split_lds_bytes(int32_t hot_groups, int32_t slices) {
  // packed bins (copies, groups, sinks), then the slice histogram with its sinks and item count
  return (size_t)(kCopySlots + (hot_groups > 0 ? hot_groups : 0) + kWave) * 8 + (size_t)(slices + kWave + 4) * 4;
}

int32_t group_split_max_hot_groups(int32_t slices, const DeviceInfo &dev) {
  const size_t fixed = group_split_lds_bytes(0, slices);
  if (dev.lds_per_block <= fixed) return 0;
  return (int32_t)((dev.lds_per_block - fixed) / 8);
}

GroupPlan group_plan(int64_t n_fact, int32_t n_groups, const DeviceInfo &dev) {
  GroupPlan pl;
  // at least 64 workgroups: every workgroup gets fewer than kPackMaxRows rows of a round
  pl.blocks = dev.cu_count > 64 ? dev.cu_count : 64;
  pl.wshift = kGroupSliceShift;
  pl.slices = (int32_t)(((int64_t)n_groups + (1 << pl.wshift) - 1) >> pl.wshift);
  pl.round = n_fact < kGroupMaxRound ? n_fact : kGroupMaxRound;
  static_assert(kGroupMaxRound / 64 + 64 < kPackMaxRows, "pass-1 bins must see fewer than 2^24 rows");
  // rows per workgroup (vector ranges round up by at most 4 rows per block,
  // plus the scalar head and tail), with a generous margin
  pl.seg_cap = 4 * (((pl.round + pl.blocks - 1) / pl.blocks + 64 + 3) / 4);
  return pl;
}

int32_t group_narrow_slices(const GroupPlan &pl) {
  return ((int64_t)pl.slices << pl.wshift) <= kNarrowMaxGroups ? pl.slices : 0;
}

size_t group_partition_bytes(const GroupPlan &pl) {
  auto r = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const int32_t Q = (pl.slices > 0 ? pl.slices : 1) + group_narrow_slices(pl);
  const size_t seg = r((size_t)pl.blocks * pl.seg_cap * 4);
  return 2 * seg                                     // pair segments (keys, values)
         + (group_narrow_slices(pl) ? seg : 0)       // narrow segments
         + r((size_t)pl.round * 2 + 16)              // slice-ordered group offsets of pairs (2 bytes)
         + r((size_t)pl.round * 4 + 16)              // slice-ordered values of pairs, and narrow items
         + r((size_t)Q * pl.blocks * 4) + r((size_t)Q * 4) + r(4) + 2 * r((size_t)pl.blocks * 4) +
         r((size_t)(Q + 1) * 4);
}

hipError_t launch_group(const int32_t *keys, const int32_t *vals, int64_t n_fact, int32_t n_groups, GroupMode mode,
                        int32_t hot_groups, const int32_t *perm, int64_t *out_sum, int64_t *out_cnt,
                        uint64_t *acc_sum, uint64_t *acc_cnt, int32_t *flag, void *part_ws, size_t part_bytes,
                        const DeviceInfo &dev, hipStream_t s) {
  if (!perm) {  // accumulate straight into the outputs
    acc_sum = reinterpret_cast<uint64_t *>(out_sum);
    acc_cnt = reinterpret_cast<uint64_t *>(out_cnt);
  }
  StageTimer st = stage_begin("group_prep", s);
  hipLaunchKernelGGL(group_prep_kernel, dim3(grid_1d(n_groups, 256, dev.cu_count * 16)), dim3(256), 0, s, acc_sum,
                     acc_cnt, n_groups, flag);
  hipError_t e = hipGetLastError();
  stage_end(st, s);
  if (e != hipSuccess) return e;
  if (n_fact > 0) {
    const GroupPlan pl = group_plan(n_fact, n_groups, dev);
    const int32_t np = group_narrow_slices(pl);
    const int32_t Q = np + pl.slices;  // rows of the shared slice table
    const bool partitioned = mode != kGroupAtomic && part_ws && n_fact >= kPartitionMinFact && pl.slices > 0 &&
                             Q <= kMaxSlices && part_bytes >= group_partition_bytes(pl);
    // t is clamped to the LDS capacity of the form that runs
    int32_t t = hot_groups;
    if (mode == kGroupRange) {
      const int32_t cap = partitioned ? group_split_max_hot_groups(Q, dev) : group_max_hot_groups(dev);
      if (t > cap) t = cap;
      if (t > n_groups) t = n_groups;
      if (t < 0) t = 0;
    } else {
      t = 0;
    }
    if (!partitioned) {
      const size_t lds =
          mode == kGroupRange ? group_lds_bytes(t) : (mode == kGroupHash ? (size_t)kHashSlots * 16 : 0);
      if (mode == kGroupRange) allow_lds(group_kernel<kGroupRange>, lds);
      if (mode == kGroupHash) allow_lds(group_kernel<kGroupHash>, lds);
      // LDS counters are 32-bit: a workgroup handles fewer than 2^31 rows per launch.
      const int64_t per_launch_max = (int64_t)dev.cu_count * (1LL << 31);
      for (int64_t off = 0; off < n_fact; off += per_launch_max) {
        const int64_t n = n_fact - off < per_launch_max ? n_fact - off : per_launch_max;
        const int64_t need = (n + 4LL * kGroupThreads - 1) / (4LL * kGroupThreads);
        const int grid = need < dev.cu_count ? (int)need : dev.cu_count;
        st = stage_begin("group_single_pass", s);
        if (mode == kGroupRange)
          hipLaunchKernelGGL(group_kernel<kGroupRange>, dim3(grid), dim3(kGroupThreads), lds, s, keys + off,
                             vals + off, n, n_groups, t, acc_sum, acc_cnt, flag);
        else if (mode == kGroupHash)
          hipLaunchKernelGGL(group_kernel<kGroupHash>, dim3(grid), dim3(kGroupThreads), lds, s, keys + off,
                             vals + off, n, n_groups, t, acc_sum, acc_cnt, flag);
        else
          hipLaunchKernelGGL(group_kernel<kGroupAtomic>, dim3(grid), dim3(kGroupThreads), lds, s, keys + off,
                             vals + off, n, n_groups, t, acc_sum, acc_cnt, flag);
        e = hipGetLastError();
        stage_end(st, s);
        if (e != hipSuccess) return e;
      }
    } else {
      auto r = [](size_t x) { return (x + 255) & ~(size_t)255; };
      char *ws = (char *)part_ws;
      int32_t *seg_k = (int32_t *)ws;
      ws += r((size_t)pl.blocks * pl.seg_cap * 4);
      int32_t *seg_v = (int32_t *)ws;
      ws += r((size_t)pl.blocks * pl.seg_cap * 4);
      int32_t *seg_n = (int32_t *)ws;
      if (np) ws += r((size_t)pl.blocks * pl.seg_cap * 4);
      uint16_t *items_k = (uint16_t *)ws;
      ws += r((size_t)pl.round * 2 + 16);
      int32_t *items_v = (int32_t *)ws;
      ws += r((size_t)pl.round * 4 + 16);
      SliceTables tab;  // both streams: narrow slices [0, np), pair slices [np, Q)
      tab.hist = (uint32_t *)ws;
      ws += r((size_t)Q * pl.blocks * 4);
      tab.row_total = (uint32_t *)ws;
      ws += r((size_t)Q * 4);
      tab.total = (uint32_t *)ws;
      ws += r(4);
      tab.seg_count = (uint32_t *)ws;  // pair items per block
      ws += r((size_t)pl.blocks * 4);
      uint32_t *seg_count_n = (uint32_t *)ws;  // narrow items per block
      ws += r((size_t)pl.blocks * 4);
      tab.slice_off = (uint32_t *)ws;
      SliceTables tab_n = tab;  // the narrow stream's view
      tab_n.seg_count = seg_count_n;
      SliceTables tab_p = tab;  // the pair stream's view
      tab_p.hist = tab.hist + (size_t)np * pl.blocks;
      tab_p.slice_off = tab.slice_off + np;
      const size_t lds1 = group_split_lds_bytes(t, Q);
      const size_t lds3 = ((size_t)12 << pl.wshift) + (size_t)(Q + 1) * 4;
      allow_lds(group_split_kernel, lds1);
      allow_lds(group_slice_kernel<false>, lds3);
      allow_lds(group_slice_kernel<true>, lds3);
      for (int64_t off = 0; off < n_fact; off += pl.round) {
        const int64_t n = n_fact - off < pl.round ? n_fact - off : pl.round;
        st = stage_begin("group_split", s);
        hipLaunchKernelGGL(group_split_kernel, dim3(pl.blocks), dim3(kGroupThreads), lds1, s, keys + off, vals + off,
                           n, n_groups, t, pl.slices, pl.wshift, np, acc_sum, acc_cnt, flag, seg_k, seg_v, seg_n,
                           pl.seg_cap, tab.seg_count, seg_count_n, tab.hist);
        e = hipGetLastError();
        stage_end(st, s);
        st = stage_begin("group_plan", s);
        if (e == hipSuccess) e = launch_partition_plan(tab, Q, pl.blocks, s);
        stage_end(st, s);
        st = stage_begin("group_scatter", s);
        // with no or few privatised groups, slice 0 of a frequency-ordered layout holds most partitioned rows
        const bool combine0 = t < kCombineBelow;
        if (e == hipSuccess && np)
          e = launch_partition_scatter_narrow(tab_n, np, pl.blocks, seg_n, pl.seg_cap, pl.wshift, items_v, s,
                                              combine0);
        if (e == hipSuccess)
          e = launch_partition_scatter(tab_p, pl.slices, pl.blocks, seg_k, seg_v, pl.seg_cap, 0, pl.wshift, items_k,
                                       items_v, s, combine0);
        stage_end(st, s);
        if (e != hipSuccess) return e;
        st = stage_begin("group_slice", s);
        if (np)
          hipLaunchKernelGGL(group_slice_kernel<true>, dim3(pl.blocks), dim3(kGroupThreads), lds3, s, items_k, items_v,
                             tab_n.slice_off, np, n_groups, 0, pl.wshift, acc_sum, acc_cnt);
        hipLaunchKernelGGL(group_slice_kernel<false>, dim3(pl.blocks), dim3(kGroupThreads), lds3, s, items_k, items_v,
                           tab_p.slice_off, pl.slices, n_groups, 0, pl.wshift, acc_sum, acc_cnt);
        e = hipGetLastError();
        stage_end(st, s);
        if (e != hipSuccess) return e;
      }
    }
  }
  if (perm) {
    st = stage_begin("unpermute", s);
    hipLaunchKernelGGL(unpermute_kernel, dim3(grid_1d(n_groups, 256, dev.cu_count * 16)), dim3(256), 0, s, acc_sum,
                       acc_cnt, perm, n_groups, out_sum, out_cnt);
    e = hipGetLastError();
    stage_end(st, s);
  }
  return e;
}

}  // namespace skew

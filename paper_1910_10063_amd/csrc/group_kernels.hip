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

// LDS layout of the range mode: hot_sum[kCopySlots + t] | hot_cnt[kCopySlots + t].
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
// Partitioned form, pass 1: hot groups into LDS bins; every other valid
// (group, value) pair appended to this workgroup's segment of the cold
// buffer and counted in its slice ((g - t) >> wshift).
// ---------------------------------------------------------------------------
struct PairSink {
  int32_t *keys, *vals;  // this workgroup's segment
  int64_t cap;
  uint32_t *count;       // LDS
  uint32_t *hist;        // LDS [P]
  int32_t wshift;
};

__device__ __forceinline__ uint32_t wave_reserve(uint32_t *count, uint32_t n) {
  uint32_t base = 0;
  const uint64_t act = __ballot(1);
  const int leader = __ffsll((unsigned long long)act) - 1;
  if (lane_id() == leader) base = atomicAdd(count, n);
  return __shfl(base, leader, kWave);
}

template <int V, bool GUARD>
__device__ __forceinline__ void group_split_batch(GroupCtx &c, const PairSink &o, const i32x4 (&x)[V],
                                                  const i32x4 (&y)[V], const bool (&valid)[V]) {
  int32_t gk[V][4], gv[V][4];
#pragma unroll
  for (int u = 0; u < V; ++u) {
    gk[u][0] = x[u].x, gk[u][1] = x[u].y, gk[u][2] = x[u].z, gk[u][3] = x[u].w;
    gv[u][0] = y[u].x, gv[u][1] = y[u].y, gv[u][2] = y[u].z, gv[u][3] = y[u].w;
  }
  bool cold[V][4];
#pragma unroll
  for (int u = 0; u < V; ++u)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int32_t g = gk[u][j];
      const bool ok = !GUARD || valid[u];
      const bool in = ok && (uint32_t)g < (uint32_t)c.m;
      if (ok && !in) c.bad = true;
      const bool h = in && g < c.t;
      cold[u][j] = in && !h;
      if (h) group_hot(c, g, gv[u][j]);
    }
  uint64_t mk[V][4];
  uint32_t total = 0;
#pragma unroll
  for (int u = 0; u < V; ++u)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      mk[u][j] = __ballot(cold[u][j]);
      total += (uint32_t)__popcll(mk[u][j]);
    }
  if (total == 0) return;
  uint32_t pos = wave_reserve(o.count, total);
  const uint64_t lt = (1ull << lane_id()) - 1ull;
#pragma unroll
  for (int u = 0; u < V; ++u)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (cold[u][j]) {
        const uint32_t idx = pos + (uint32_t)__popcll(mk[u][j] & lt);
        if (idx < o.cap) {
          o.keys[idx] = gk[u][j];
          o.vals[idx] = gv[u][j];
        }
        lds_add_u32(&o.hist[(uint32_t)(gk[u][j] - c.t) >> o.wshift], 1u);
      }
      pos += (uint32_t)__popcll(mk[u][j]);
    }
}

__device__ __forceinline__ void group_split_one(GroupCtx &c, const PairSink &o, bool valid, int32_t g, int32_t v) {
  const bool in = valid && (uint32_t)g < (uint32_t)c.m;
  if (valid && !in) c.bad = true;
  const bool h = in && g < c.t;
  const bool cd = in && !h;
  if (h) group_hot(c, g, v);
  const uint64_t m = __ballot(cd);
  if (m) {
    const uint32_t base = wave_reserve(o.count, (uint32_t)__popcll(m));
    if (cd) {
      const uint32_t idx = base + (uint32_t)__popcll(m & ((1ull << lane_id()) - 1ull));
      if (idx < o.cap) {
        o.keys[idx] = g;
        o.vals[idx] = v;
      }
      lds_add_u32(&o.hist[(uint32_t)(g - c.t) >> o.wshift], 1u);
    }
  }
}

__global__ __launch_bounds__(kGroupThreads) void group_split_kernel(
    const int32_t *__restrict__ keys, const int32_t *__restrict__ vals, int64_t n, int32_t m, int32_t t, int32_t P,
    int32_t wshift, uint64_t *__restrict__ acc_sum, uint64_t *__restrict__ acc_cnt, int32_t *flag,
    int32_t *__restrict__ seg_keys, int32_t *__restrict__ seg_vals, int64_t seg_cap, uint32_t *__restrict__ seg_count,
    uint32_t *__restrict__ hist) {
  extern __shared__ __align__(16) unsigned char smem[];
  GroupCtx c;
  c.m = m;
  c.t = t;
  c.ncopy = t < kGroupCopies ? t : kGroupCopies;
  c.acc_sum = acc_sum;
  c.acc_cnt = acc_cnt;
  c.bad = false;
  group_range_init(c, smem, t);
  uint32_t *lhist = c.hot_cnt + kCopySlots + t;
  uint32_t *lcount = lhist + P;
  for (int p = threadIdx.x; p < P; p += blockDim.x) lhist[p] = 0;
  if (threadIdx.x == 0) *lcount = 0;
  __syncthreads();
  PairSink o;
  o.keys = seg_keys + (int64_t)blockIdx.x * seg_cap;
  o.vals = seg_vals + (int64_t)blockIdx.x * seg_cap;
  o.cap = seg_cap;
  o.count = lcount;
  o.hist = lhist;
  o.wshift = wshift;

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
      group_split_one(c, o, i >= 0, i >= 0 ? keys[i] : 0, i >= 0 ? vals[i] : 0);
    }
    const int64_t per = (sp.nvec + gridDim.x - 1) / gridDim.x;
    const int64_t vb = (int64_t)blockIdx.x * per < sp.nvec ? (int64_t)blockIdx.x * per : sp.nvec;
    const int64_t ve = vb + per < sp.nvec ? vb + per : sp.nvec;
    const i32x4 *vk = reinterpret_cast<const i32x4 *>(keys + sp.head);
    const i32x4 *vv = reinterpret_cast<const i32x4 *>(vals + sp.head);
    const int64_t tile_vecs = (int64_t)kGroupThreads * kGroupUnroll;
    const bool all_valid[kGroupUnroll] = {true, true};
    for (int64_t base = vb; base < ve; base += tile_vecs) {
      i32x4 x[kGroupUnroll], y[kGroupUnroll];
      if (base + tile_vecs <= ve) {
#pragma unroll
        for (int u = 0; u < kGroupUnroll; ++u) {
          x[u] = load_stream4(vk + base + u * kGroupThreads + threadIdx.x);
          y[u] = load_stream4(vv + base + u * kGroupThreads + threadIdx.x);
        }
        group_split_batch<kGroupUnroll, false>(c, o, x, y, all_valid);
      } else {
        bool valid[kGroupUnroll];
#pragma unroll
        for (int u = 0; u < kGroupUnroll; ++u) {
          const int64_t vi = base + u * kGroupThreads + threadIdx.x;
          valid[u] = vi < ve;
          x[u] = valid[u] ? load_stream4(vk + vi) : i32x4{0, 0, 0, 0};
          y[u] = valid[u] ? load_stream4(vv + vi) : i32x4{0, 0, 0, 0};
        }
        group_split_batch<kGroupUnroll, true>(c, o, x, y, valid);
      }
    }
  } else {
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t rb = (int64_t)blockIdx.x * per < n ? (int64_t)blockIdx.x * per : n;
    const int64_t re = rb + per < n ? rb + per : n;
    for (int64_t base = rb; base < re; base += blockDim.x) {
      const int64_t i = base + threadIdx.x;
      const bool valid = i < re;
      group_split_one(c, o, valid, valid ? load_stream1(keys + i) : 0, valid ? load_stream1(vals + i) : 0);
    }
  }
  if (c.bad) *flag = 1;
  __syncthreads();
  if (threadIdx.x == 0) seg_count[blockIdx.x] = *lcount < seg_cap ? *lcount : (uint32_t)seg_cap;
  for (int p = threadIdx.x; p < P; p += blockDim.x) hist[(int64_t)p * gridDim.x + blockIdx.x] = lhist[p];
  group_range_flush(c);
}

// ---------------------------------------------------------------------------
// Partitioned form, pass 3: the (group, value) pairs of each unit are summed
// in LDS bins of their slice (W groups); the bins are flushed into the shared
// accumulators when the workgroup moves to another slice and at the end.
// ---------------------------------------------------------------------------
constexpr int kSliceUnroll = 8;

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

__global__ __launch_bounds__(kGroupThreads) void group_slice_kernel(
    const int32_t *__restrict__ keys, const int32_t *__restrict__ vals, const uint32_t *__restrict__ slice_off,
    const uint32_t *__restrict__ unit_start, int32_t P, int32_t m, int32_t t, int32_t wshift,
    uint64_t *__restrict__ acc_sum, uint64_t *__restrict__ acc_cnt) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int32_t W = 1 << wshift;
  uint64_t *bsum = reinterpret_cast<uint64_t *>(smem);
  uint32_t *bcnt = reinterpret_cast<uint32_t *>(bsum + W);
  uint32_t *ustart = bcnt + W;
  uint32_t *soff = ustart + (P + 1);
  for (int i = threadIdx.x; i < W; i += blockDim.x) {
    bsum[i] = 0;
    bcnt[i] = 0;
  }
  for (int p = threadIdx.x; p <= P; p += blockDim.x) {
    ustart[p] = unit_start[p];
    soff[p] = slice_off[p];
  }
  __syncthreads();
  const uint32_t units = ustart[P];
  const uint32_t u0 = (uint32_t)((uint64_t)units * blockIdx.x / gridDim.x);
  const uint32_t u1 = (uint32_t)((uint64_t)units * (blockIdx.x + 1) / gridDim.x);
  int32_t p = 0, cur = -1;
  int64_t cur_base = 0;
  int32_t cur_len = 0;
  for (uint32_t u = u0; u < u1; ++u) {
    while (p + 1 < P && ustart[p + 1] <= u) ++p;
    if (p != cur) {
      if (cur >= 0) {
        __syncthreads();
        slice_flush(bsum, bcnt, cur_len, cur_base, acc_sum, acc_cnt);
      }
      cur = p;
      cur_base = (int64_t)t + ((int64_t)p << wshift);
      cur_len = (int32_t)((int64_t)m - cur_base < W ? (int64_t)m - cur_base : W);
      __syncthreads();
    }
    const uint32_t lo = soff[p] + (u - ustart[p]) * kUnitItems;
    const uint32_t hi = lo + kUnitItems < soff[p + 1] ? lo + kUnitItems : soff[p + 1];
    const uint32_t smax = (uint32_t)cur_len - 1;
    constexpr uint32_t kChunk = kSliceUnroll * kGroupThreads;
    uint32_t i = lo + threadIdx.x;
    const uint32_t full = lo + ((hi - lo) / kChunk) * kChunk;
    int32_t g[kSliceUnroll], v[kSliceUnroll], gn[kSliceUnroll], vn[kSliceUnroll];
    auto load = [&](int32_t(&gg)[kSliceUnroll], int32_t(&vv)[kSliceUnroll], uint32_t at) {
#pragma unroll
      for (int j = 0; j < kSliceUnroll; ++j) {
        gg[j] = load_stream1(keys + at + j * kGroupThreads);
        vv[j] = load_stream1(vals + at + j * kGroupThreads);
      }
    };
    if (i < full) load(g, v, i);
    for (; i < full; i += kChunk) {
      load(gn, vn, i + kChunk < full ? i + kChunk : i);
#pragma unroll
      for (int j = 0; j < kSliceUnroll; ++j) {
        uint32_t local = (uint32_t)(g[j] - (int32_t)cur_base);
        local = local < smax ? local : smax;
        lds_add_u64(&bsum[local], (uint64_t)(int64_t)v[j]);
        lds_add_u32(&bcnt[local], 1u);
      }
#pragma unroll
      for (int j = 0; j < kSliceUnroll; ++j) {
        g[j] = gn[j];
        v[j] = vn[j];
      }
    }
    for (; i < hi; i += kGroupThreads) {
      uint32_t local = (uint32_t)(load_stream1(keys + i) - (int32_t)cur_base);
      local = local < smax ? local : smax;
      lds_add_u64(&bsum[local], (uint64_t)(int64_t)load_stream1(vals + i));
      lds_add_u32(&bcnt[local], 1u);
    }
  }
  if (cur >= 0) {
    __syncthreads();
    slice_flush(bsum, bcnt, cur_len, cur_base, acc_sum, acc_cnt);
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
  const size_t fixed = group_lds_bytes(0) + (size_t)(kMaxSlices + 4) * 4;  // + slice histogram of pass 1
  if (dev.lds_per_block <= fixed) return 0;
  return (int32_t)((dev.lds_per_block - fixed) / 12);
}

GroupPlan group_plan(int64_t n_fact, int32_t n_groups, int32_t t, const DeviceInfo &dev) {
  GroupPlan pl;
  pl.blocks = dev.cu_count > 0 ? dev.cu_count : 256;
  pl.wshift = kGroupSliceShift;
  const int64_t cold = (int64_t)n_groups - t;
  pl.slices = cold > 0 ? (int32_t)((cold + (1 << pl.wshift) - 1) >> pl.wshift) : 0;
  pl.round = n_fact < kMaxRound ? n_fact : kMaxRound;
  // rows per workgroup (vector ranges round up by at most 4 rows per block,
  // plus the scalar head and tail), with a generous margin
  pl.seg_cap = 4 * (((pl.round + pl.blocks - 1) / pl.blocks + 64 + 3) / 4);
  return pl;
}

size_t group_partition_bytes(const GroupPlan &pl) {
  auto r = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const int32_t P = pl.slices > 0 ? pl.slices : 1;
  return 2 * r((size_t)pl.blocks * pl.seg_cap * 4)  // cold segments (keys, values)
         + 2 * r((size_t)pl.round * 4 + 16)         // slice-ordered pairs
         + r((size_t)P * pl.blocks * 4) + r((size_t)P * 4) + r(4) + r((size_t)pl.blocks * 4) + 2 * r((size_t)(P + 1) * 4);
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
    int32_t t = hot_groups;
    if (mode == kGroupRange) {
      const int32_t cap = group_max_hot_groups(dev);
      if (t > cap) t = cap;
      if (t > n_groups) t = n_groups;
      if (t < 0) t = 0;
    } else {
      t = 0;
    }
    const GroupPlan pl = group_plan(n_fact, n_groups, t, dev);
    const bool partitioned = mode != kGroupAtomic && part_ws && n_fact >= kPartitionMinFact && pl.slices > 0 &&
                             pl.slices <= kMaxSlices && part_bytes >= group_partition_bytes(pl);
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
      int32_t *items_k = (int32_t *)ws;
      ws += r((size_t)pl.round * 4 + 16);
      int32_t *items_v = (int32_t *)ws;
      ws += r((size_t)pl.round * 4 + 16);
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
      tab.unit_start = (uint32_t *)ws;
      const size_t lds1 = group_lds_bytes(t) + (size_t)(pl.slices + 4) * 4;
      const size_t lds3 = ((size_t)12 << pl.wshift) + (size_t)2 * (pl.slices + 1) * 4;
      allow_lds(group_split_kernel, lds1);
      allow_lds(group_slice_kernel, lds3);
      for (int64_t off = 0; off < n_fact; off += pl.round) {
        const int64_t n = n_fact - off < pl.round ? n_fact - off : pl.round;
        st = stage_begin("group_split", s);
        hipLaunchKernelGGL(group_split_kernel, dim3(pl.blocks), dim3(kGroupThreads), lds1, s, keys + off, vals + off,
                           n, n_groups, t, pl.slices, pl.wshift, acc_sum, acc_cnt, flag, seg_k, seg_v, pl.seg_cap,
                           tab.seg_count, tab.hist);
        e = hipGetLastError();
        stage_end(st, s);
        st = stage_begin("group_plan", s);
        if (e == hipSuccess) e = launch_partition_plan(tab, pl.slices, pl.blocks, s);
        stage_end(st, s);
        st = stage_begin("group_scatter", s);
        if (e == hipSuccess)
          e = launch_partition_scatter(tab, pl.slices, pl.blocks, seg_k, seg_v, pl.seg_cap, t, pl.wshift, items_k,
                                       items_v, s);
        stage_end(st, s);
        if (e != hipSuccess) return e;
        st = stage_begin("group_slice", s);
        hipLaunchKernelGGL(group_slice_kernel, dim3(pl.blocks), dim3(kGroupThreads), lds3, s, items_k, items_v,
                           tab.slice_off, tab.unit_start, pl.slices, n_groups, t, pl.wshift, acc_sum, acc_cnt);
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

// Query kernels: FK join-aggregate with a hot dimension prefix in LDS
// (Section 4.2: threshold-based processing) and grouped aggregation with
// private hot groups and shared cold groups (Section 4.3, Section 4.2.2).
#include "device_common.h"
#include "kernels.h"

namespace skew {
namespace {

// ---------------------------------------------------------------------------
// Per-query dimension word.  Section 3.2 builds, for each query, a copy of
// the dimension columns it needs in layout order; here the two columns the
// query needs (price, category) and its predicate are packed into one 32-bit
// word per row, so a fact row costs one 4-byte gather:
//   0x80000000 | (g + 1) << 25 | price   qualifies, group g, 0 <= price < 2^25
//   0x80000000                           does not qualify (or has no group)
//   0                                    qualifies, but the price does not fit:
//                                        the slow path reads the columns again
// A gather outside [0, n_rows) also reads 0 (buffer range check), so every
// zero word goes to the slow path, which tells the two cases apart.  Field
// (w >> 25) & 31 selects an accumulator bin; bin 0 is a sink that is never
// read back.
// ---------------------------------------------------------------------------
constexpr uint32_t kValid = 0x80000000u;
constexpr int kGroupShift = 25;
constexpr uint32_t kPriceMask = (1u << kGroupShift) - 1u;

__device__ __forceinline__ bool row_group(int32_t c, int32_t cat_lt, int32_t by_cat, int32_t *g) {
  if (!(c < cat_lt)) return false;
  if (by_cat) {
    if (c < 0 || c >= 16) return false;
    *g = c;
  } else {
    *g = 0;
  }
  return true;
}

__global__ void join_pack_kernel(const int32_t *__restrict__ price, const int8_t *__restrict__ cat, int32_t n_rows,
                                 int32_t cat_lt, int32_t by_cat, uint32_t *__restrict__ words,
                                 int64_t *__restrict__ out_sum, int64_t *__restrict__ out_cnt, int32_t *flag) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid < (by_cat ? 16 : 1)) {
    out_sum[gid] = 0;
    out_cnt[gid] = 0;
  }
  if (gid == 0) *flag = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = gid; r < n_rows; r += stride) {
    const int32_t p = price[r];
    int32_t g;
    uint32_t w = kValid;
    if (row_group(cat[r], cat_lt, by_cat, &g))
      w = ((uint32_t)p <= kPriceMask) ? (kValid | ((uint32_t)(g + 1) << kGroupShift) | (uint32_t)p) : 0u;
    words[r] = w;
  }
}

// Structured buffer load: element `index` of a buffer of 4-byte records.  The
// hardware range check (index < num_records) returns 0 for any other index,
// negative keys included, without touching memory.
typedef int32_t rsrc_t __attribute__((ext_vector_type(4)));
__device__ uint32_t buffer_load_record(rsrc_t rsrc, int32_t vindex, int32_t voffset, int32_t soffset,
                                       int32_t aux) __asm("llvm.amdgcn.struct.buffer.load.i32");

__device__ __forceinline__ rsrc_t record_buffer(const void *base, uint32_t num_records) {
  const uint64_t a = (uint64_t)(uintptr_t)base;
  rsrc_t r;
  r.x = (int32_t)(uint32_t)a;
  r.y = (int32_t)(((uint32_t)(a >> 32) & 0xFFFFu) | (4u << 16));  // stride 4 bytes
  r.z = (int32_t)num_records;
  r.w = 0x00020000;  // gfx9 raw 32-bit data format
  return r;
}

// Join-aggregate.  One workgroup of 1024 threads per CU; dimension rows
// [0, t_lds) are copied into LDS once per workgroup (Section 4.2.1: ids below
// the threshold are the likely cache hits and take their own path).  Every
// fact key is looked up twice without branching: a clamped LDS read and a
// buffer gather whose index is pushed out of range for hot keys (so it
// returns 0 and issues no memory traffic); a select keeps the right one.
// For GROUPS == 16 every lane owns one 64-bit bin per group in LDS, shared by
// the 16 waves through LDS atomics (two lanes of a wave never hit the same
// bin); a bin packs count << 44 | sum, exact while it sees fewer than 2^19
// rows.  For GROUPS == 1 the sums stay in registers.
constexpr int kJoinVecs = 4;  // 16-byte key vectors per lane per batch
constexpr int kJoinBins = 32;  // (w >> 25) & 31
constexpr int kCountShift = 44;
constexpr uint64_t kSumMask = (1ull << kCountShift) - 1ull;

template <int GROUPS>
struct JoinCtx {
  const uint32_t *hot;  // LDS
  uint64_t *bins;       // LDS [kJoinBins][64], GROUPS == 16
  rsrc_t words;
  uint32_t t, tclamp;
  uint32_t lane8;
  // GROUPS == 1
  uint64_t sum;
  uint32_t cnt;
  // slow path
  const int32_t *price;
  const int8_t *cat;
  int32_t cat_lt;
  uint32_t n_rows;
  int64_t *out_sum, *out_cnt;
  bool bad;
};

template <int GROUPS>
__device__ __forceinline__ uint32_t join_fetch(const JoinCtx<GROUPS> &c, uint32_t uk) {
  const bool h = uk < c.t;
  const uint32_t wl = c.hot[uk < c.tclamp ? uk : c.tclamp];
  const uint32_t wg = buffer_load_record(c.words, (int32_t)(h ? 0xFFFFFFFFu : uk), 0, 0, 0);
  return h ? wl : wg;
}

template <int GROUPS>
__device__ __forceinline__ void join_slow(JoinCtx<GROUPS> &c, uint32_t uk) {
  if (uk >= c.n_rows) {
    c.bad = true;
    return;
  }
  int32_t g;
  if (row_group(c.cat[uk], c.cat_lt, GROUPS == 16, &g)) {
    global_add_u64(reinterpret_cast<uint64_t *>(&c.out_sum[g]), (uint64_t)(int64_t)c.price[uk]);
    global_add_u64(reinterpret_cast<uint64_t *>(&c.out_cnt[g]), 1ull);
  }
}

// One batch of 4 * V keys: all gathers first, then all accumulations.
template <int GROUPS, int V>
__device__ __forceinline__ void join_batch(JoinCtx<GROUPS> &c, const i32x4 (&x)[V]) {
  uint32_t w[V][4];
#pragma unroll
  for (int u = 0; u < V; ++u) {
    w[u][0] = join_fetch(c, (uint32_t)x[u].x);
    w[u][1] = join_fetch(c, (uint32_t)x[u].y);
    w[u][2] = join_fetch(c, (uint32_t)x[u].z);
    w[u][3] = join_fetch(c, (uint32_t)x[u].w);
  }
  uint32_t all = kValid;
  uint32_t s32 = 0, c32 = 0;
#pragma unroll
  for (int u = 0; u < V; ++u) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t wj = w[u][j];
      all &= wj;
      if (GROUPS == 16) {
        const uint32_t bin = (wj >> kGroupShift) & (kJoinBins - 1);
        lds_add_u64(&c.bins[bin * kWave + lane_id()], (1ull << kCountShift) | (wj & kPriceMask));
      } else {
        s32 += wj & kPriceMask;
        c32 += (wj >> kGroupShift) & 1u;
      }
    }
  }
  if (GROUPS == 1) {
    c.sum += s32;
    c.cnt += c32;
  }
  if (__builtin_expect(!(all & kValid), 0)) {  // an escape or out-of-range key in this batch
#pragma unroll
    for (int u = 0; u < V; ++u) {
      if (!w[u][0]) join_slow(c, (uint32_t)x[u].x);
      if (!w[u][1]) join_slow(c, (uint32_t)x[u].y);
      if (!w[u][2]) join_slow(c, (uint32_t)x[u].z);
      if (!w[u][3]) join_slow(c, (uint32_t)x[u].w);
    }
  }
}

template <int GROUPS>
__device__ __forceinline__ void join_single(JoinCtx<GROUPS> &c, int32_t k) {
  const uint32_t w = join_fetch(c, (uint32_t)k);
  if (GROUPS == 16) {
    lds_add_u64(&c.bins[((w >> kGroupShift) & (kJoinBins - 1)) * kWave + lane_id()],
                (1ull << kCountShift) | (w & kPriceMask));
  } else {
    c.sum += w & kPriceMask;
    c.cnt += (w >> kGroupShift) & 1u;
  }
  if (!w) join_slow(c, (uint32_t)k);
}

template <int GROUPS>
__global__ __launch_bounds__(kJoinThreads) void join_kernel(const int32_t *__restrict__ keys, int64_t n,
                                                            const uint32_t *__restrict__ words, int32_t n_rows,
                                                            int32_t t_lds, const int32_t *__restrict__ price,
                                                            const int8_t *__restrict__ cat, int32_t cat_lt,
                                                            int64_t *__restrict__ out_sum,
                                                            int64_t *__restrict__ out_cnt, int32_t *flag) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int kBinBytes = GROUPS == 16 ? kJoinBins * kWave * 8 : 0;
  JoinCtx<GROUPS> c;
  c.bins = reinterpret_cast<uint64_t *>(smem);
  uint32_t *hot = reinterpret_cast<uint32_t *>(smem + kBinBytes);
  c.hot = hot;
  c.words = record_buffer(words, (uint32_t)n_rows);
  c.t = (uint32_t)t_lds;
  c.tclamp = t_lds > 0 ? (uint32_t)t_lds - 1 : 0u;  // LDS always holds at least one word
  c.sum = 0;
  c.cnt = 0;
  c.price = price;
  c.cat = cat;
  c.cat_lt = cat_lt;
  c.n_rows = (uint32_t)n_rows;
  c.out_sum = out_sum;
  c.out_cnt = out_cnt;
  c.bad = false;
  if (GROUPS == 16)
    for (int i = threadIdx.x; i < kJoinBins * kWave; i += blockDim.x) c.bins[i] = 0;
  {  // stage the hot prefix (words is 256-byte aligned workspace)
    const int nv = t_lds >> 2;
    const uint4 *src = reinterpret_cast<const uint4 *>(words);
    uint4 *dst = reinterpret_cast<uint4 *>(hot);
    for (int i = threadIdx.x; i < nv; i += blockDim.x) dst[i] = src[i];
    for (int i = 4 * nv + threadIdx.x; i < t_lds; i += blockDim.x) hot[i] = words[i];
    if (t_lds == 0 && threadIdx.x == 0) hot[0] = 0;
  }
  __syncthreads();

  const Split4 sp = split4(keys, n);
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid < sp.head) join_single(c, keys[gid]);
  if (gid < n - sp.tail) join_single(c, keys[sp.tail + gid]);

  // Full tiles of kJoinThreads * kJoinVecs vectors, two batches in flight:
  // the next tile's keys are loaded while the current one is processed.
  const i32x4 *vk = reinterpret_cast<const i32x4 *>(keys + sp.head);
  const int64_t tile_vecs = (int64_t)kJoinThreads * kJoinVecs;
  const int64_t ntiles = sp.nvec / tile_vecs;
  int64_t tile = blockIdx.x;
  i32x4 xa[kJoinVecs], xb[kJoinVecs];
  auto load_tile = [&](i32x4(&x)[kJoinVecs], int64_t tl) {
    const i32x4 *p = vk + tl * tile_vecs + threadIdx.x;
#pragma unroll
    for (int u = 0; u < kJoinVecs; ++u) x[u] = load_stream4(p + u * kJoinThreads);
  };
  // The prefetch is unconditional (the last one re-reads the current tile) so
  // that every path has the same loads in flight and the wait before a batch
  // covers only that batch's keys.
  if (tile < ntiles) load_tile(xa, tile);
  while (tile < ntiles) {
    int64_t nxt = tile + gridDim.x;
    load_tile(xb, nxt < ntiles ? nxt : tile);
    join_batch<GROUPS, kJoinVecs>(c, xa);
    tile = nxt;
    if (tile >= ntiles) break;
    nxt = tile + gridDim.x;
    load_tile(xa, nxt < ntiles ? nxt : tile);
    join_batch<GROUPS, kJoinVecs>(c, xb);
    tile = nxt;
  }
  for (int64_t v = ntiles * tile_vecs + gid; v < sp.nvec; v += (int64_t)gridDim.x * blockDim.x) {
    const i32x4 x[1] = {load_stream4(vk + v)};
    join_batch<GROUPS, 1>(c, x);
  }
  if (c.bad) *flag = 1;

  // Workgroup reduction, then one global atomic per group.
  if (GROUPS == 1) {
    __shared__ uint64_t red_s[kJoinThreads / kWave];
    __shared__ uint32_t red_c[kJoinThreads / kWave];
    const uint64_t s = wave_sum_u64(c.sum);
    const uint32_t k = wave_sum_u32(c.cnt);
    const int w = threadIdx.x / kWave;
    if (lane_id() == 0) {
      red_s[w] = s;
      red_c[w] = k;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      uint64_t ts = 0, tc = 0;
      for (int i = 0; i < (int)(blockDim.x / kWave); ++i) {
        ts += red_s[i];
        tc += red_c[i];
      }
      if (tc) {
        global_add_u64(reinterpret_cast<uint64_t *>(&out_sum[0]), ts);
        global_add_u64(reinterpret_cast<uint64_t *>(&out_cnt[0]), tc);
      }
    }
  } else {
    __syncthreads();
    const int g = threadIdx.x / kWave;  // 16 waves <-> 16 groups, bin g + 1
    if (g < 16) {
      const uint64_t e = c.bins[(g + 1) * kWave + lane_id()];
      const uint64_t s = wave_sum_u64(e & kSumMask);
      const uint64_t k = wave_sum_u64(e >> kCountShift);
      if (lane_id() == 0 && k) {
        global_add_u64(reinterpret_cast<uint64_t *>(&out_sum[g]), s);
        global_add_u64(reinterpret_cast<uint64_t *>(&out_cnt[g]), k);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Grouped aggregation
// ---------------------------------------------------------------------------
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
  int32_t t;      // range mode: groups [0, t) live in LDS
  int32_t ncopy;  // range mode: groups [0, ncopy) have per-lane copies, ncopy = min(t, kGroupCopies)
  uint64_t *acc_sum;
  uint64_t *acc_cnt;
  bool bad;
  // range mode
  uint64_t *copy_sum;  // [kGroupCopies][64]
  uint32_t *copy_cnt;
  uint64_t *bin_sum;   // [t]
  uint32_t *bin_cnt;
  // hash mode
  int32_t *slot_key;   // [kHashSlots]
  uint64_t *slot_sum;
  uint32_t *slot_cnt;
};

__device__ __forceinline__ void group_global(const GroupCtx &c, int32_t g, int32_t v) {
  global_add_u64(&c.acc_sum[g], (uint64_t)(int64_t)v);
  global_add_u64(&c.acc_cnt[g], 1ull);
}

template <int MODE>
__device__ __forceinline__ void group_one(GroupCtx &c, int32_t g, int32_t v) {
  if ((uint32_t)g >= (uint32_t)c.m) {
    c.bad = true;
    return;
  }
  if (MODE == kGroupRange) {
    if (g < c.ncopy) {  // hottest groups: one copy per lane, never contended within a wave
      const int i = g * kWave + lane_id();
      lds_add_u64(&c.copy_sum[i], (uint64_t)(int64_t)v);
      lds_add_u32(&c.copy_cnt[i], 1u);
    } else if (g < c.t) {
      lds_add_u64(&c.bin_sum[g], (uint64_t)(int64_t)v);
      lds_add_u32(&c.bin_cnt[g], 1u);
    } else {
      group_global(c, g, v);
    }
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
    c.copy_sum = reinterpret_cast<uint64_t *>(smem);
    c.bin_sum = c.copy_sum + kGroupCopies * kWave;
    c.copy_cnt = reinterpret_cast<uint32_t *>(c.bin_sum + t);
    c.bin_cnt = c.copy_cnt + kGroupCopies * kWave;
    for (int i = threadIdx.x; i < kGroupCopies * kWave; i += blockDim.x) {
      c.copy_sum[i] = 0;
      c.copy_cnt[i] = 0;
    }
    for (int i = threadIdx.x; i < t; i += blockDim.x) {
      c.bin_sum[i] = 0;
      c.bin_cnt[i] = 0;
    }
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

  // Flush the private bins into the shared accumulators.
  if (MODE == kGroupRange) {
    const int w = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;
    for (int g = w; g < c.ncopy; g += nw) {
      const uint64_t s = wave_sum_u64(c.copy_sum[g * kWave + lane_id()]);
      const uint64_t k = wave_sum_u64((uint64_t)c.copy_cnt[g * kWave + lane_id()]);
      if (lane_id() == 0 && k) {
        global_add_u64(&acc_sum[g], s);
        global_add_u64(&acc_cnt[g], k);
      }
    }
    for (int g = kGroupCopies + threadIdx.x; g < t; g += blockDim.x) {
      const uint32_t k = c.bin_cnt[g];
      if (k) {
        global_add_u64(&acc_sum[g], c.bin_sum[g]);
        global_add_u64(&acc_cnt[g], (uint64_t)k);
      }
    }
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

// Allow dynamic LDS up to the device limit (above the 64 KB default).
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
size_t join_lds_bytes(int groups, int32_t hot_rows) {
  const size_t hot = hot_rows > 0 ? ((size_t)hot_rows * 4 + 15) & ~(size_t)15 : 16;
  return (groups == 16 ? (size_t)kJoinBins * kWave * 8 : 0) + hot;
}

int32_t join_max_hot_rows(int groups, const DeviceInfo &dev) {
  const size_t fixed = join_lds_bytes(groups, 0) - 16 + 256;  // bins + static reduction scratch
  if (dev.lds_per_block <= fixed) return 0;
  return (int32_t)(((dev.lds_per_block - fixed) / 4) & ~(size_t)3);
}

size_t group_lds_bytes(int32_t hot_groups) {
  return (size_t)kGroupCopies * kWave * 12 + (size_t)hot_groups * 12;
}

int32_t group_max_hot_groups(const DeviceInfo &dev) {
  const size_t fixed = group_lds_bytes(0);
  if (dev.lds_per_block <= fixed) return 0;
  return (int32_t)((dev.lds_per_block - fixed) / 12);
}

hipError_t launch_join(const int32_t *keys, int64_t n_fact, const int32_t *price, const int8_t *cat, int32_t n_rows,
                       int32_t cat_lt, int32_t by_cat, int32_t hot_rows, int64_t *out_sum, int64_t *out_cnt,
                       uint32_t *words, int32_t *flag, const DeviceInfo &dev, hipStream_t s) {
  const int groups = by_cat ? 16 : 1;
  hipLaunchKernelGGL(join_pack_kernel, dim3(grid_1d(n_rows > 16 ? n_rows : 16, 256, dev.cu_count * 16)), dim3(256), 0,
                     s, price, cat, n_rows, cat_lt, by_cat, words, out_sum, out_cnt, flag);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || n_fact == 0) return e;
  int32_t t = hot_rows;
  const int32_t cap = join_max_hot_rows(groups, dev);
  if (t > cap) t = cap;
  if (t > n_rows) t = n_rows;
  if (t < 0) t = 0;
  const size_t lds = join_lds_bytes(groups, t);
  // Every lane's bins must see fewer than 2^18 rows per launch: at most 16
  // waves share a bin, so a thread handles at most 2^14 rows per launch.
  const int64_t per_launch_max = (int64_t)dev.cu_count * kJoinThreads * (1LL << 14);
  for (int64_t off = 0; off < n_fact; off += per_launch_max) {
    const int64_t n = n_fact - off < per_launch_max ? n_fact - off : per_launch_max;
    const int64_t need = (n + 4LL * kJoinThreads - 1) / (4LL * kJoinThreads);
    const int grid = need < dev.cu_count ? (int)need : dev.cu_count;
    if (groups == 16) allow_lds(join_kernel<16>, lds);
    else allow_lds(join_kernel<1>, lds);
    if (groups == 16)
      hipLaunchKernelGGL(join_kernel<16>, dim3(grid), dim3(kJoinThreads), lds, s, keys + off, n, words, n_rows, t,
                         price, cat, cat_lt, out_sum, out_cnt, flag);
    else
      hipLaunchKernelGGL(join_kernel<1>, dim3(grid), dim3(kJoinThreads), lds, s, keys + off, n, words, n_rows, t,
                         price, cat, cat_lt, out_sum, out_cnt, flag);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_group(const int32_t *keys, const int32_t *vals, int64_t n_fact, int32_t n_groups, GroupMode mode,
                        int32_t hot_groups, const int32_t *perm, int64_t *out_sum, int64_t *out_cnt,
                        uint64_t *acc_sum, uint64_t *acc_cnt, int32_t *flag, const DeviceInfo &dev, hipStream_t s) {
  if (!perm) {  // accumulate straight into the outputs
    acc_sum = reinterpret_cast<uint64_t *>(out_sum);
    acc_cnt = reinterpret_cast<uint64_t *>(out_cnt);
  }
  hipLaunchKernelGGL(group_prep_kernel, dim3(grid_1d(n_groups, 256, dev.cu_count * 16)), dim3(256), 0, s, acc_sum,
                     acc_cnt, n_groups, flag);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (n_fact > 0) {
    int32_t t = hot_groups;
    if (mode == kGroupRange) {
      const int32_t cap = group_max_hot_groups(dev);
      if (t > cap) t = cap;
      if (t > n_groups) t = n_groups;
      if (t < 0) t = 0;
    }
    const size_t lds = mode == kGroupRange ? group_lds_bytes(t) : (mode == kGroupHash ? (size_t)kHashSlots * 16 : 0);
    // LDS counters are 32-bit: a workgroup handles fewer than 2^31 rows per launch.
    const int64_t per_launch_max = (int64_t)dev.cu_count * (1LL << 31);
    for (int64_t off = 0; off < n_fact; off += per_launch_max) {
      const int64_t n = n_fact - off < per_launch_max ? n_fact - off : per_launch_max;
      const int64_t need = (n + 4LL * kGroupThreads - 1) / (4LL * kGroupThreads);
      const int grid = need < dev.cu_count ? (int)need : dev.cu_count;
      if (mode == kGroupRange) allow_lds(group_kernel<kGroupRange>, lds);
      if (mode == kGroupHash) allow_lds(group_kernel<kGroupHash>, lds);
      if (mode == kGroupRange)
        hipLaunchKernelGGL(group_kernel<kGroupRange>, dim3(grid), dim3(kGroupThreads), lds, s, keys + off, vals + off,
                           n, n_groups, t, acc_sum, acc_cnt, flag);
      else if (mode == kGroupHash)
        hipLaunchKernelGGL(group_kernel<kGroupHash>, dim3(grid), dim3(kGroupThreads), lds, s, keys + off, vals + off,
                           n, n_groups, t, acc_sum, acc_cnt, flag);
      else
        hipLaunchKernelGGL(group_kernel<kGroupAtomic>, dim3(grid), dim3(kGroupThreads), lds, s, keys + off,
                           vals + off, n, n_groups, t, acc_sum, acc_cnt, flag);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  }
  if (perm) {
    hipLaunchKernelGGL(unpermute_kernel, dim3(grid_1d(n_groups, 256, dev.cu_count * 16)), dim3(256), 0, s, acc_sum,
                       acc_cnt, perm, n_groups, out_sum, out_cnt);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace skew

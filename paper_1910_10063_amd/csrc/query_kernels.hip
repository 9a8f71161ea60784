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
//   0                     row does not qualify (or has no group)
//   0x40000000 | g << 26 | price   qualifies, group g, 0 <= price < 2^26
//   0x80000000            qualifies but the price does not fit: read the
//                         columns again (exact for any int32 price)
// ---------------------------------------------------------------------------
constexpr uint32_t kQualifies = 0x40000000u;
constexpr uint32_t kEscape = 0x80000000u;
constexpr uint32_t kPriceMask = (1u << 26) - 1u;

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
    uint32_t w = 0;
    if (row_group(cat[r], cat_lt, by_cat, &g))
      w = ((uint32_t)p <= kPriceMask) ? (kQualifies | ((uint32_t)g << 26) | (uint32_t)p) : kEscape;
    words[r] = w;
  }
}

// Join-aggregate.  One workgroup of 1024 threads per CU; dimension rows
// [0, t_lds) are copied into LDS once per workgroup.  For GROUPS == 16 every
// lane owns one 64-bit bin per group in LDS, shared by the 16 waves through
// LDS atomics (no two lanes of a wave ever hit the same bin); a bin packs
// count << 44 | sum, exact while a bin sees fewer than 2^18 rows.
constexpr int kJoinUnroll = 4;
constexpr int kCountShift = 44;
constexpr uint64_t kSumMask = (1ull << kCountShift) - 1ull;

template <int GROUPS>
struct JoinAcc {
  uint64_t sum = 0;
  uint32_t cnt = 0;
  uint64_t *bins = nullptr;
};

template <int GROUPS>
__device__ __forceinline__ void join_consume(JoinAcc<GROUPS> &acc, uint32_t w, int32_t k, const int32_t *price,
                                             const int8_t *cat, int32_t cat_lt, int64_t *out_sum,
                                             int64_t *out_cnt) {
  if (w & kEscape) {  // rare: price outside [0, 2^26)
    int32_t g;
    if (row_group(cat[k], cat_lt, GROUPS == 16, &g)) {
      global_add_u64(reinterpret_cast<uint64_t *>(&out_sum[g]), (uint64_t)(int64_t)price[k]);
      global_add_u64(reinterpret_cast<uint64_t *>(&out_cnt[g]), 1ull);
    }
    return;
  }
  if (!(w & kQualifies)) return;
  const uint32_t p = w & kPriceMask;
  if (GROUPS == 1) {
    acc.sum += p;
    acc.cnt += 1;
  } else {
    const uint32_t g = (w >> 26) & 15u;
    lds_add_u64(&acc.bins[g * kWave + lane_id()], (1ull << kCountShift) | p);
  }
}

template <int GROUPS>
__global__ __launch_bounds__(kJoinThreads) void join_kernel(const int32_t *__restrict__ keys, int64_t n,
                                                            const uint32_t *__restrict__ words, int32_t n_rows,
                                                            int32_t t_lds, const int32_t *__restrict__ price,
                                                            const int8_t *__restrict__ cat, int32_t cat_lt,
                                                            int64_t *__restrict__ out_sum,
                                                            int64_t *__restrict__ out_cnt, int32_t *flag) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int kBinBytes = GROUPS == 16 ? 16 * kWave * 8 : 0;
  uint32_t *hot = reinterpret_cast<uint32_t *>(smem + kBinBytes);
  JoinAcc<GROUPS> acc;
  if (GROUPS == 16) {
    acc.bins = reinterpret_cast<uint64_t *>(smem);
    for (int i = threadIdx.x; i < 16 * kWave; i += blockDim.x) acc.bins[i] = 0;
  }
  {  // stage the hot prefix (words is 256-byte aligned workspace)
    const int nv = t_lds >> 2;
    const uint4 *src = reinterpret_cast<const uint4 *>(words);
    uint4 *dst = reinterpret_cast<uint4 *>(hot);
    for (int i = threadIdx.x; i < nv; i += blockDim.x) dst[i] = src[i];
    for (int i = 4 * nv + threadIdx.x; i < t_lds; i += blockDim.x) hot[i] = words[i];
  }
  __syncthreads();

  auto lookup = [&](int32_t k, uint32_t &w) -> bool {
    if ((uint32_t)k < (uint32_t)t_lds) {
      w = hot[k];
    } else if ((uint32_t)k < (uint32_t)n_rows) {
      w = words[k];
    } else {
      raise_flag(flag);
      return false;
    }
    return true;
  };
  auto one = [&](int32_t k) {
    uint32_t w;
    if (lookup(k, w)) join_consume<GROUPS>(acc, w, k, price, cat, cat_lt, out_sum, out_cnt);
  };

  const Split4 sp = split4(keys, n);
  const int64_t T = (int64_t)gridDim.x * blockDim.x;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid < sp.head) one(keys[gid]);
  if (gid < n - sp.tail) one(keys[sp.tail + gid]);
  const i32x4 *vk = reinterpret_cast<const i32x4 *>(keys + sp.head);
  int64_t v = gid;
  for (; v + (kJoinUnroll - 1) * T < sp.nvec; v += kJoinUnroll * T) {
    i32x4 x[kJoinUnroll];
#pragma unroll
    for (int u = 0; u < kJoinUnroll; ++u) x[u] = load_stream4(vk + v + u * T);
    uint32_t w[kJoinUnroll][4];
    bool ok[kJoinUnroll][4];
#pragma unroll
    for (int u = 0; u < kJoinUnroll; ++u) {
      ok[u][0] = lookup(x[u].x, w[u][0]);
      ok[u][1] = lookup(x[u].y, w[u][1]);
      ok[u][2] = lookup(x[u].z, w[u][2]);
      ok[u][3] = lookup(x[u].w, w[u][3]);
    }
#pragma unroll
    for (int u = 0; u < kJoinUnroll; ++u) {
      if (ok[u][0]) join_consume<GROUPS>(acc, w[u][0], x[u].x, price, cat, cat_lt, out_sum, out_cnt);
      if (ok[u][1]) join_consume<GROUPS>(acc, w[u][1], x[u].y, price, cat, cat_lt, out_sum, out_cnt);
      if (ok[u][2]) join_consume<GROUPS>(acc, w[u][2], x[u].z, price, cat, cat_lt, out_sum, out_cnt);
      if (ok[u][3]) join_consume<GROUPS>(acc, w[u][3], x[u].w, price, cat, cat_lt, out_sum, out_cnt);
    }
  }
  for (; v < sp.nvec; v += T) {
    const i32x4 x = load_stream4(vk + v);
    one(x.x);
    one(x.y);
    one(x.z);
    one(x.w);
  }

  // Workgroup reduction, then one global atomic per group.
  if (GROUPS == 1) {
    __shared__ uint64_t red_s[kJoinThreads / kWave];
    __shared__ uint32_t red_c[kJoinThreads / kWave];
    const uint64_t s = wave_sum_u64(acc.sum);
    const uint32_t c = wave_sum_u32(acc.cnt);
    const int w = threadIdx.x / kWave;
    if (lane_id() == 0) {
      red_s[w] = s;
      red_c[w] = c;
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
    const int g = threadIdx.x / kWave;  // 16 waves <-> 16 groups
    if (g < 16) {
      const uint64_t e = acc.bins[g * kWave + lane_id()];
      const uint64_t s = wave_sum_u64(e & kSumMask);
      const uint64_t c = wave_sum_u64(e >> kCountShift);
      if (lane_id() == 0 && c) {
        global_add_u64(reinterpret_cast<uint64_t *>(&out_sum[g]), s);
        global_add_u64(reinterpret_cast<uint64_t *>(&out_cnt[g]), c);
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
  int32_t *flag;
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
__device__ __forceinline__ void group_one(const GroupCtx &c, int32_t g, int32_t v) {
  if ((uint32_t)g >= (uint32_t)c.m) {
    raise_flag(c.flag);
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
  c.flag = flag;
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
  return (groups == 16 ? 16 * kWave * 8 : 0) + (size_t)hot_rows * 4;
}

int32_t join_max_hot_rows(int groups, const DeviceInfo &dev) {
  const size_t fixed = join_lds_bytes(groups, 0) + 256;  // static reduction scratch
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

// FK join-aggregate (Q1/Q2 of Section 1 feeding SUM/COUNT) with
// threshold-based processing (Section 4.2): dimension rows [0, t) are copied
// into LDS once per workgroup and keys below t are resolved there.  Keys at or
// above t are either gathered from global memory (single pass) or written to
// a cold buffer, partitioned by dimension slice and resolved from LDS copies
// of the slices in a second pass (the threshold split of Section 4.2.1).
#include "kernels.h"
#include "profiler.h"
#include "query_common.h"

namespace skew {
namespace {

__global__ void join_pack_kernel(const int32_t *__restrict__ price, const int8_t *__restrict__ cat, int32_t n_rows,
                                 int32_t cat_lt, int32_t by_cat, uint32_t *__restrict__ words,
                                 int64_t *__restrict__ out_sum, int64_t *__restrict__ out_cnt, int32_t *flag) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid < (by_cat ? 16 : 1)) {
    out_sum[gid] = 0;
    out_cnt[gid] = 0;
  }
  if (gid == 0) *flag = 0;
  auto pack = [&](int32_t p, int32_t c) -> uint32_t {
    int32_t g;
    if (!row_group(c, cat_lt, by_cat, &g)) return kValid;
    return ((uint32_t)p <= kPriceMask) ? (kValid | ((uint32_t)(g + 1) << kGroupShift) | (uint32_t)p) : 0u;
  };
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t done = 0;  // rows [0, done) packed four at a time
  if ((((uintptr_t)price & 15u) | ((uintptr_t)cat & 3u) | ((uintptr_t)words & 15u)) == 0) {
    const int64_t nv = n_rows / 4;
    const i32x4 *p4 = reinterpret_cast<const i32x4 *>(price);
    const uint32_t *c4 = reinterpret_cast<const uint32_t *>(cat);
    uint4 *w4 = reinterpret_cast<uint4 *>(words);
    for (int64_t v = gid; v < nv; v += stride) {
      const i32x4 p = load_stream4(p4 + v);
      const uint32_t c = c4[v];
      w4[v] = uint4{pack(p.x, (int8_t)c), pack(p.y, (int8_t)(c >> 8)), pack(p.z, (int8_t)(c >> 16)),
                    pack(p.w, (int8_t)(c >> 24))};
    }
    done = 4 * nv;
  }
  for (int64_t r = done + gid; r < n_rows; r += stride) words[r] = pack(price[r], cat[r]);
}

constexpr int kJoinVecs = 4;  // 16-byte key vectors per lane per batch
constexpr int64_t kJoinAutoMinHot = 8192;  // smallest automatic prefix of the single pass


// Accumulators.  GROUPS == 16: every lane owns one 64-bit bin per group in
// LDS, shared by the 16 waves of the workgroup through LDS atomics (two lanes
// of a wave never hit the same bin); a bin packs count << 44 | sum and stays
// exact while it sees fewer than 2^19 rows (enforced per launch).
// GROUPS == 1: sums in registers.
template <int GROUPS>
struct JoinCtx {
  uint64_t *bins;  // LDS [kJoinBinRows][64]
  uint64_t sum;
  uint32_t cnt;
  bool bad;
  // slow path (price outside [0, 2^25) or key outside the dimension)
  const int32_t *price;
  const int8_t *cat;
  int32_t cat_lt;
  uint32_t n_rows;
  int64_t *out_sum, *out_cnt;
};

template <int GROUPS>
__device__ __forceinline__ void join_init(JoinCtx<GROUPS> &c, unsigned char *smem, const int32_t *price,
                                          const int8_t *cat, int32_t cat_lt, int32_t n_rows, int64_t *out_sum,
                                          int64_t *out_cnt) {
  c.bins = reinterpret_cast<uint64_t *>(smem);
  c.sum = 0;
  c.cnt = 0;
  c.bad = false;
  c.price = price;
  c.cat = cat;
  c.cat_lt = cat_lt;
  c.n_rows = (uint32_t)n_rows;
  c.out_sum = out_sum;
  c.out_cnt = out_cnt;
  if (GROUPS == 16)
    for (int i = threadIdx.x; i < kJoinBinRows * kWave; i += blockDim.x) c.bins[i] = 0;
}

template <int GROUPS>
__device__ __forceinline__ void join_add(JoinCtx<GROUPS> &c, uint32_t w) {
  if (GROUPS == 16) {
    const uint32_t bin = (w >> kGroupShift) & (kJoinBins - 1);
    lds_add_u64(&c.bins[bin * kWave + lane_id()], (1ull << kCountShift) | (w & kPriceMask));
  } else {
    c.sum += w & kPriceMask;
    c.cnt += (w >> kGroupShift) & 1u;
  }
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

// The rare slow path of a batch: one loop over its slots instead of a copy
// of join_slow per slot, so the common path stays small.
template <int GROUPS, int N>
__device__ __forceinline__ void join_slow_batch(JoinCtx<GROUPS> &c, const uint32_t (&w)[N], const uint32_t (&k)[N]) {
#pragma unroll 1
  for (int s = 0; s < N; ++s) {
    uint32_t ws = w[0], ks = k[0];
#pragma unroll
    for (int q = 1; q < N; ++q) {
      ws = s == q ? w[q] : ws;
      ks = s == q ? k[q] : ks;
    }
    if (!ws) join_slow(c, ks);
  }
}

// Workgroup reduction of the accumulators, then one global atomic per group.
template <int GROUPS>
__device__ __forceinline__ void join_flush(JoinCtx<GROUPS> &c, int32_t *flag) {
  if (c.bad) *flag = 1;
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
        global_add_u64(reinterpret_cast<uint64_t *>(&c.out_sum[0]), ts);
        global_add_u64(reinterpret_cast<uint64_t *>(&c.out_cnt[0]), tc);
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
        global_add_u64(reinterpret_cast<uint64_t *>(&c.out_sum[g]), s);
        global_add_u64(reinterpret_cast<uint64_t *>(&c.out_cnt[g]), k);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Single pass: one workgroup of 1024 threads per CU, grid-stride over tiles of
// 1024 x kJoinVecs key vectors, the next tile loaded while the current one is
// processed.
// ---------------------------------------------------------------------------
template <int GROUPS, int V>
__device__ __forceinline__ void join_batch(JoinCtx<GROUPS> &c, const HotCtx &h, const i32x4 (&x)[V]) {
  uint32_t k[4 * V], w[4 * V];
#pragma unroll
  for (int u = 0; u < V; ++u) {
    k[4 * u] = (uint32_t)x[u].x, k[4 * u + 1] = (uint32_t)x[u].y;
    k[4 * u + 2] = (uint32_t)x[u].z, k[4 * u + 3] = (uint32_t)x[u].w;
  }
#pragma unroll
  for (int i = 0; i < 4 * V; ++i) w[i] = fetch_hot_or_global(h, k[i]);
  uint32_t all = kValid;
#pragma unroll
  for (int i = 0; i < 4 * V; ++i) {
    all &= w[i];
    join_add(c, w[i]);
  }
  if (__builtin_expect(!(all & kValid), 0)) join_slow_batch(c, w, k);  // an escape or out-of-range key
}

template <int GROUPS>
__device__ __forceinline__ void join_single(JoinCtx<GROUPS> &c, const HotCtx &h, int32_t k) {
  const uint32_t w = fetch_hot_or_global(h, (uint32_t)k);
  join_add(c, w);
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
  constexpr int kBinBytes = GROUPS == 16 ? kJoinBinRows * kWave * 8 : 0;
  JoinCtx<GROUPS> c;
  join_init(c, smem, price, cat, cat_lt, n_rows, out_sum, out_cnt);
  uint32_t *hot = reinterpret_cast<uint32_t *>(smem + kBinBytes);
  HotCtx h;
  h.hot = hot;
  h.words = record_buffer(words, (uint32_t)n_rows);
  h.t = (uint32_t)t_lds;
  h.tclamp = t_lds > 0 ? (uint32_t)t_lds - 1 : 0u;  // LDS always holds at least one word

  // Tiles of kJoinVecs vectors per thread while every workgroup gets at least
  // one; below that (small inputs) one vector per thread, so that all
  // workgroups share the keys.  The first keys are requested before the
  // prefix is staged, so that a workgroup waits for both at once.  The tile
  // prefetch is unconditional (the last one re-reads the current tile) so
  // that every path has the same loads in flight and the wait before a batch
  // covers only that batch's keys.
  const Split4 sp = split4(keys, n);
  const i32x4 *vk = reinterpret_cast<const i32x4 *>(keys + sp.head);
  const int64_t tile_vecs = (int64_t)kJoinThreads * kJoinVecs;
  const int64_t ntiles = sp.nvec / tile_vecs >= (int64_t)gridDim.x ? sp.nvec / tile_vecs : 0;
  int64_t tile = blockIdx.x;
  i32x4 xa[kJoinVecs], xb[kJoinVecs];
  auto load_tile = [&](i32x4(&x)[kJoinVecs], int64_t tl) {
    const i32x4 *p = vk + tl * tile_vecs + threadIdx.x;
#pragma unroll
    for (int u = 0; u < kJoinVecs; ++u) x[u] = load_stream4(p + u * kJoinThreads);
  };
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t vstride = (int64_t)gridDim.x * blockDim.x;
  int64_t v = ntiles * tile_vecs + gid;  // this thread's first single vector
  i32x4 x1 = {0, 0, 0, 0};
  if (tile < ntiles) load_tile(xa, tile);
  else if (v < sp.nvec) x1 = load_stream4(vk + v);
  stage_words(hot, words, 0, t_lds);
  if (t_lds == 0 && threadIdx.x == 0) hot[0] = 0;
  __syncthreads();

  if (gid < sp.head) join_single(c, h, keys[gid]);
  if (gid < n - sp.tail) join_single(c, h, keys[sp.tail + gid]);

  while (tile < ntiles) {
    int64_t nxt = tile + gridDim.x;
    load_tile(xb, nxt < ntiles ? nxt : tile);
    join_batch<GROUPS, kJoinVecs>(c, h, xa);
    tile = nxt;
    if (tile >= ntiles) break;
    nxt = tile + gridDim.x;
    load_tile(xa, nxt < ntiles ? nxt : tile);
    join_batch<GROUPS, kJoinVecs>(c, h, xb);
    tile = nxt;
  }
  if (ntiles > 0 && v < sp.nvec) x1 = load_stream4(vk + v);
  for (; v < sp.nvec; v += vstride) {
    const i32x4 x[1] = {x1};
    if (v + vstride < sp.nvec) x1 = load_stream4(vk + v + vstride);  // the next vector, while this one is resolved
    join_batch<GROUPS, 1>(c, h, x);
  }
  join_flush(c, flag);
}

// ---------------------------------------------------------------------------
// Partitioned form, pass 1: keys below t_lds are resolved from LDS; keys in
// [t, tail_start) are appended to this workgroup's segment of the cold
// buffer and counted in their slice ((k - t) >> wshift).  Workgroup b owns a
// contiguous range of the column, so its segment needs no more slots than
// the rows it reads.  With GATHER, the other keys inside the dimension are
// gathered from global memory as in the single pass: the warm rows
// [t_lds, t) of a threshold t beyond the LDS capacity (hot in the paper's
// sense, held by the caches instead of LDS), and the tail [tail_start,
// n_rows) of a dimension with more cold rows than kMaxSlices slices.
// ---------------------------------------------------------------------------
struct Tail {
  uint32_t start;  // first row past the slices (n_rows without a tail)
  rsrc_t words;    // all dimension words, range-checked
  uint32_t t_lds;  // rows [0, t_lds) are in LDS; rows [t_lds, t) are gathered
};

template <int GROUPS, int V, bool GUARD, bool GATHER>
__device__ __forceinline__ void join_split_batch(JoinCtx<GROUPS> &c, const ColdSink &o, rsrc_t seg,
                                                 const uint32_t *hot, uint32_t tclamp, const Tail &tail,
                                                 const i32x4 (&x)[V], const bool (&valid)[V]) {
  uint32_t k[4 * V], w[4 * V];
  bool cold[4 * V];
#pragma unroll
  for (int u = 0; u < V; ++u) {
    k[4 * u] = (uint32_t)x[u].x, k[4 * u + 1] = (uint32_t)x[u].y;
    k[4 * u + 2] = (uint32_t)x[u].z, k[4 * u + 3] = (uint32_t)x[u].w;
  }
#pragma unroll
  for (int i = 0; i < 4 * V; ++i) {
    const bool ok = !GUARD || valid[i / 4];
    const bool h = ok && k[i] < (GATHER ? tail.t_lds : o.t);
    cold[i] = GATHER ? ok && k[i] >= o.t && k[i] < tail.start : ok && !h && k[i] < c.n_rows;
    c.bad |= ok && k[i] >= c.n_rows;
    const uint32_t wl = hot[k[i] < tclamp ? k[i] : tclamp];
    w[i] = h ? wl : kValid;
    if (GATHER) {  // warm and tail keys; an out-of-range index for every other key: no memory traffic
      const bool gl = ok && !h && !cold[i] && k[i] < c.n_rows;
      const uint32_t wg = buffer_load_record(tail.words, (int32_t)(gl ? k[i] : 0xFFFFFFFFu), 0, 0, 0);
      w[i] = gl ? wg : w[i];
    }
  }
  uint32_t all = kValid;
#pragma unroll
  for (int i = 0; i < 4 * V; ++i) {
    all &= w[i];
    join_add(c, w[i]);
  }
  if (__builtin_expect(!(all & kValid), 0)) join_slow_batch(c, w, k);  // a hot row whose price escapes
  auto st = [&](int i, int32_t idx) { buffer_store_record((int32_t)k[i], seg, idx, 0, 0, 0); };
  cold_append<4 * V, decltype(st), true>(o, k, cold, st);
}

template <int GROUPS>
__device__ __forceinline__ void join_split_one(JoinCtx<GROUPS> &c, const ColdSink &o, rsrc_t seg,
                                               const uint32_t *hot, uint32_t tclamp, const Tail &tail, bool valid,
                                               uint32_t k) {
  const bool h = valid && k < tail.t_lds;
  const bool cold = valid && k >= o.t && k < tail.start;
  const bool gl = valid && !h && !cold && k < c.n_rows;  // warm or tail
  const uint32_t wg = buffer_load_record(tail.words, (int32_t)(gl ? k : 0xFFFFFFFFu), 0, 0, 0);
  const uint32_t w = h ? hot[k < tclamp ? k : tclamp] : (gl ? wg : kValid);
  c.bad |= valid && k >= c.n_rows;
  join_add(c, w);
  if (!w) join_slow(c, k);
  const uint32_t kk[1] = {k};
  const bool cd[1] = {cold};
  cold_append(o, kk, cd, [&](int, int32_t idx) { buffer_store_record((int32_t)k, seg, idx, 0, 0, 0); });
}

template <int GROUPS, bool GATHER>
__global__ __launch_bounds__(kJoinThreads) void join_split_kernel(
    const int32_t *__restrict__ keys, int64_t n, const uint32_t *__restrict__ words, int32_t n_rows, int32_t t_lds,
    int32_t t, int32_t P, int32_t wshift, int32_t tail_start, const int32_t *__restrict__ price, const int8_t *__restrict__ cat, int32_t cat_lt,
    int64_t *__restrict__ out_sum, int64_t *__restrict__ out_cnt, int32_t *flag, int32_t *__restrict__ cold_seg,
    int64_t seg_cap, uint32_t *__restrict__ seg_count, uint32_t *__restrict__ hist) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int kBinBytes = GROUPS == 16 ? kJoinBinRows * kWave * 8 : 0;
  JoinCtx<GROUPS> c;
  join_init(c, smem, price, cat, cat_lt, n_rows, out_sum, out_cnt);
  uint32_t *hot = reinterpret_cast<uint32_t *>(smem + kBinBytes);
  const int32_t hot_words = (t_lds + 4) & ~3;  // at least one word, 16-byte multiple
  uint32_t *lhist = hot + hot_words;
  uint32_t *lcount = lhist + P + kWave;
  stage_words(hot, words, 0, t_lds);
  if (t_lds == 0 && threadIdx.x == 0) hot[0] = 0;
  for (int p = threadIdx.x; p < P + kWave; p += blockDim.x) lhist[p] = 0;
  if (threadIdx.x == 0) *lcount = 0;
  __syncthreads();

  const rsrc_t seg = record_buffer(cold_seg + (int64_t)blockIdx.x * seg_cap, (uint32_t)seg_cap);
  ColdSink o;
  o.count = lcount;
  o.hist = lhist;
  o.t = (uint32_t)t;  // first partitioned row
  o.wshift = wshift;
  o.sink = (uint32_t)P + lane_id();
  // with no or a small hot prefix, slice 0 of a frequency-ordered layout takes most cold keys: its lanes are
  // counted once per slot instead of queueing on one counter
  o.combine0 = t < kCombineBelow;
  const uint32_t tclamp = t_lds > 0 ? (uint32_t)t_lds - 1 : 0u;
  const Tail tail{(uint32_t)tail_start, record_buffer(words, (uint32_t)n_rows), (uint32_t)t_lds};

  // Contiguous range of key vectors per workgroup; block 0 takes the scalar
  // head, the last block the scalar tail.
  const Split4 sp = split4(keys, n);
  const int64_t per = (sp.nvec + gridDim.x - 1) / gridDim.x;
  const int64_t vb = (int64_t)blockIdx.x * per < sp.nvec ? (int64_t)blockIdx.x * per : sp.nvec;
  const int64_t ve = vb + per < sp.nvec ? vb + per : sp.nvec;
  {  // scalar head (block 0, lanes 0-2) and tail (last block, lanes 64-66)
    int64_t i = -1;
    if (blockIdx.x == 0 && threadIdx.x < sp.head) i = threadIdx.x;
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x >= 64 && threadIdx.x - 64 < n - sp.tail)
      i = sp.tail + threadIdx.x - 64;
    join_split_one(c, o, seg, hot, tclamp, tail, i >= 0, i >= 0 ? (uint32_t)keys[i] : 0u);
  }

  const i32x4 *vk = reinterpret_cast<const i32x4 *>(keys + sp.head);
  const int64_t tile_vecs = (int64_t)kJoinThreads * kJoinVecs;
  const int64_t full_end = vb + ((ve - vb) / tile_vecs) * tile_vecs;
  const bool all_valid[kJoinVecs] = {true, true, true, true};
  auto load_tile = [&](i32x4(&x)[kJoinVecs], int64_t base) {
    const i32x4 *p = vk + base + threadIdx.x;
#pragma unroll
    for (int u = 0; u < kJoinVecs; ++u) x[u] = load_stream4(p + u * kJoinThreads);
  };
  i32x4 xa[kJoinVecs], xb[kJoinVecs];
  int64_t base = vb;
  if (base < full_end) load_tile(xa, base);
  while (base < full_end) {
    int64_t nxt = base + tile_vecs;
    load_tile(xb, nxt < full_end ? nxt : base);
    join_split_batch<GROUPS, kJoinVecs, false, GATHER>(c, o, seg, hot, tclamp, tail, xa, all_valid);
    base = nxt;
    if (base >= full_end) break;
    nxt = base + tile_vecs;
    load_tile(xa, nxt < full_end ? nxt : base);
    join_split_batch<GROUPS, kJoinVecs, false, GATHER>(c, o, seg, hot, tclamp, tail, xb, all_valid);
    base = nxt;
  }
  if (full_end < ve) {  // last partial tile
    i32x4 x[kJoinVecs];
    bool valid[kJoinVecs];
#pragma unroll
    for (int u = 0; u < kJoinVecs; ++u) {
      const int64_t vi = full_end + u * kJoinThreads + threadIdx.x;
      valid[u] = vi < ve;
      x[u] = valid[u] ? load_stream4(vk + vi) : i32x4{0, 0, 0, 0};
    }
    join_split_batch<GROUPS, kJoinVecs, true, GATHER>(c, o, seg, hot, tclamp, tail, x, valid);
  }
  __syncthreads();
  if (threadIdx.x == 0) seg_count[blockIdx.x] = *lcount < seg_cap ? *lcount : (uint32_t)seg_cap;
  for (int p = threadIdx.x; p < P; p += blockDim.x) hist[(int64_t)p * gridDim.x + blockIdx.x] = lhist[p];
  join_flush(c, flag);
}

// ---------------------------------------------------------------------------
// Partitioned form, pass 3: the slice-ordered cold items (2-byte offsets
// inside their slice) are cut into one contiguous share per workgroup,
// balanced over items plus the cost of copying each slice; the workgroup
// walks the slices its share touches, copies each into LDS when its part of
// the slice is large enough to pay for the copy, and gathers the words from
// global memory otherwise.
// ---------------------------------------------------------------------------
constexpr int kSliceVecs = 2;  // 16-byte vectors (8 items each) per lane per batch

template <bool DENSE>
struct SliceLookup {
  const uint32_t *slice;  // LDS copy of rows [sbase, sbase + W)
  uint32_t sbase;
  rsrc_t words;
  __device__ __forceinline__ uint32_t operator()(uint32_t local) const {
    if (DENSE) return slice[local];
    return buffer_load_record(words, (int32_t)(sbase + local), 0, 0, 0);
  }
};

template <int GROUPS, int V, class L>
__device__ __forceinline__ void join_slice_batch(JoinCtx<GROUPS> &c, const L &look, const i32x4 (&x)[V],
                                                 const bool (&valid)[V]) {
  uint32_t l[8 * V], w[8 * V];
#pragma unroll
  for (int u = 0; u < V; ++u) {
    const uint32_t d[4] = {(uint32_t)x[u].x, (uint32_t)x[u].y, (uint32_t)x[u].z, (uint32_t)x[u].w};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      l[8 * u + 2 * j] = d[j] & 0xFFFFu;
      l[8 * u + 2 * j + 1] = d[j] >> 16;
    }
  }
#pragma unroll
  for (int i = 0; i < 8 * V; ++i) w[i] = valid[i / 8] ? look(l[i]) : kValid;
  uint32_t all = kValid;
#pragma unroll
  for (int i = 0; i < 8 * V; ++i) {
    all &= w[i];
    join_add(c, w[i]);
  }
  if (__builtin_expect(!(all & kValid), 0)) {
#pragma unroll
    for (int i = 0; i < 8 * V; ++i) l[i] += look.sbase;  // back to dimension rows for the slow path
    join_slow_batch(c, w, l);
  }
}

template <int GROUPS, class L>
__device__ __forceinline__ void join_slice_range(JoinCtx<GROUPS> &c, const L &look, const uint16_t *__restrict__ items,
                                                 uint32_t lo, uint32_t hi) {
  const i32x4 *vk = reinterpret_cast<const i32x4 *>(items);
  walk_items<8, kSliceVecs, kJoinThreads, i32x4>(
      lo, hi,
      [&](uint32_t i) {
        const uint32_t local = items[i];
        const uint32_t w = look(local);
        join_add(c, w);
        if (!w) join_slow(c, look.sbase + local);
      },
      [&](uint32_t vi) { return load_stream4(vk + vi); },
      [&](const i32x4(&x)[kSliceVecs], const bool(&valid)[kSliceVecs]) {
        join_slice_batch<GROUPS, kSliceVecs>(c, look, x, valid);
      });
}

template <int GROUPS>
__global__ __launch_bounds__(kJoinThreads) void join_slice_kernel(
    const uint16_t *__restrict__ items, const uint32_t *__restrict__ slice_off, int32_t P,
    const uint32_t *__restrict__ words, int32_t n_rows, int32_t t, int32_t wshift, const int32_t *__restrict__ price,
    const int8_t *__restrict__ cat, int32_t cat_lt, int64_t *__restrict__ out_sum, int64_t *__restrict__ out_cnt,
    int32_t *flag) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int kBinBytes = GROUPS == 16 ? kJoinBinRows * kWave * 8 : 0;
  JoinCtx<GROUPS> c;
  join_init(c, smem, price, cat, cat_lt, n_rows, out_sum, out_cnt);
  const int32_t W = 1 << wshift;
  uint32_t *slice = reinterpret_cast<uint32_t *>(smem + kBinBytes);
  uint32_t *soff = slice + W;
  for (int p = threadIdx.x; p <= P; p += blockDim.x) soff[p] = slice_off[p];
  __syncthreads();
  const rsrc_t wr = record_buffer(words, (uint32_t)n_rows);
  // copying a slice moves 4 W bytes, as much as 2 W items of 2 bytes
  uint32_t lo, hi;
  balanced_share(soff, P, 2u * (uint32_t)W, blockIdx.x, gridDim.x, &lo, &hi);
  int32_t p = lo < hi ? slice_of_item(soff, P, lo) : P;
  for (uint32_t at = lo; at < hi; ++p) {
    const uint32_t end = soff[p + 1] < hi ? soff[p + 1] : hi;
    if (end <= at) continue;
    const int64_t sbase = (int64_t)t + ((int64_t)p << wshift);
    const int32_t slen = (int32_t)((int64_t)n_rows - sbase < W ? (int64_t)n_rows - sbase : W);
    if (end - at >= (uint32_t)(W >> 3)) {  // enough items to pay for copying the slice
      __syncthreads();
      stage_words(slice, words, sbase, slen);
      __syncthreads();
      const SliceLookup<true> look{slice, (uint32_t)sbase, wr};
      join_slice_range(c, look, items, at, end);
    } else {
      const SliceLookup<false> look{slice, (uint32_t)sbase, wr};
      join_slice_range(c, look, items, at, end);
    }
    at = end;
  }
  join_flush(c, flag);
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
size_t join_lds_bytes(int groups, int32_t hot_rows) {
  const size_t hot = (((size_t)(hot_rows > 0 ? hot_rows : 0) + 4) & ~(size_t)3) * 4;
  return (groups == 16 ? (size_t)kJoinBinRows * kWave * 8 : 0) + hot;
}

int32_t join_max_hot_rows(int groups, const DeviceInfo &dev) {
  // bins + static reduction scratch + slice histogram of the partitioned form
  const size_t fixed = join_lds_bytes(groups, 0) - 16 + 256 + (size_t)(kMaxSlices + kWave + 4) * 4;
  if (dev.lds_per_block <= fixed) return 0;
  return (int32_t)(((dev.lds_per_block - fixed) / 4) & ~(size_t)3) - 4;
}

JoinPlan join_plan(int64_t n_fact, int32_t n_rows, int32_t t, int groups, const DeviceInfo &dev) {
  JoinPlan pl;
  // at least 32 workgroups, so that no accumulator bin sees 2^19 rows of a round (a bin takes the rows of one
  // lane position of a workgroup: fewer than 2^29 / 32 / 64 = 2^18 rows)
  pl.blocks = dev.cu_count > 32 ? dev.cu_count : 32;
  static_assert(kJoinMaxRound / 32 / kWave + 64 < (1LL << 19), "join bins must see fewer than 2^19 rows");
  pl.wshift = kJoinSliceShift;
  const int64_t cold_rows = (int64_t)n_rows - t;
  pl.slices = cold_rows > 0 ? (int32_t)((cold_rows + (1 << pl.wshift) - 1) >> pl.wshift) : 0;
  if (pl.slices > kMaxSlices) pl.slices = kMaxSlices;  // rows past the last slice are gathered (the tail)
  pl.round = n_fact < kJoinMaxRound ? n_fact : kJoinMaxRound;
  const int64_t nvec = (pl.round + 3) / 4 + 1;
  pl.seg_cap = 4 * ((nvec + pl.blocks - 1) / pl.blocks) + 8;
  (void)groups;
  return pl;
}

size_t join_partition_bytes(const JoinPlan &pl) {
  auto r = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const int32_t P = pl.slices > 0 ? pl.slices : 1;
  return r((size_t)pl.blocks * pl.seg_cap * 4)       // cold segments
         + r((size_t)pl.round * 2 + 16)              // slice-ordered items (2-byte offsets)
         + r((size_t)P * pl.blocks * 4)              // (slice, block) counts
         + r((size_t)P * 4) + r(4) + r((size_t)pl.blocks * 4) + r((size_t)(P + 1) * 4);
}

int32_t join_hot_rows_used(int64_t n_fact, int32_t n_rows, int32_t by_cat, int32_t hot_rows, size_t part_bytes,
                           const DeviceInfo &dev, bool *partitioned) {
  const int groups = by_cat ? 16 : 1;
  const int32_t cap = join_max_hot_rows(groups, dev);
  int32_t t = hot_rows < 0 ? cap : hot_rows;
  if (t > n_rows) t = n_rows;
  const int32_t tc = t < cap ? t : cap;
  // the workspace holds the partitioned form's buffers for the threshold clamped to LDS (they do not grow
  // with a warm range); a threshold past the last row leaves nothing to partition
  const JoinPlan pl = join_plan(n_fact, n_rows, tc, groups, dev);
  *partitioned = part_bytes > 0 && n_fact >= kPartitionMinFact && pl.slices > 0 && t < n_rows &&
                 part_bytes >= join_partition_bytes(pl);
  // rows past the LDS capacity stay hot only in the partitioned form (gathered in pass 1); the single pass
  // gathers every key past its LDS prefix anyway
  if (!*partitioned) t = tc;
  if (!*partitioned && hot_rows < 0) {
    // Every workgroup of the single pass copies the prefix into LDS: for a small input, a prefix much longer
    // than half the keys a workgroup reads costs more to stage than its lookups save (8192 rows at 1e6-4e6
    // keys).
    const int64_t per_launch_max = (int64_t)dev.cu_count * kJoinThreads * (1LL << 14);
    const int64_t n0 = n_fact < per_launch_max ? n_fact : per_launch_max;
    const int64_t need = (n0 + 4LL * kJoinThreads - 1) / (4LL * kJoinThreads);
    const int64_t per_wg = n0 / (need < dev.cu_count ? need : dev.cu_count);
    const int64_t ta = per_wg / 2 > kJoinAutoMinHot ? per_wg / 2 : kJoinAutoMinHot;
    if (ta < t) t = (int32_t)ta;
  }
  return t;
}

hipError_t launch_join(const int32_t *keys, int64_t n_fact, const int32_t *price, const int8_t *cat, int32_t n_rows,
                       int32_t cat_lt, int32_t by_cat, int32_t hot_rows, int64_t *out_sum, int64_t *out_cnt,
                       uint32_t *words, int32_t *flag, void *part_ws, size_t part_bytes, const DeviceInfo &dev,
                       hipStream_t s) {
  const int groups = by_cat ? 16 : 1;
  StageTimer st = stage_begin("join_pack", s);
  hipLaunchKernelGGL(join_pack_kernel, dim3(grid_1d(n_rows / 4 > 16 ? n_rows / 4 : 16, 256, dev.cu_count * 16)), dim3(256), 0,
                     s, price, cat, n_rows, cat_lt, by_cat, words, out_sum, out_cnt, flag);
  hipError_t e = hipGetLastError();
  stage_end(st, s);
  if (e != hipSuccess || n_fact == 0) return e;
  bool partitioned = false;
  const int32_t t = join_hot_rows_used(n_fact, n_rows, by_cat, hot_rows, part_ws ? part_bytes : 0, dev, &partitioned);
  const int32_t cap = join_max_hot_rows(groups, dev);
  const int32_t t_lds = t < cap ? t : cap;  // rows [t_lds, t) are warm: gathered in pass 1
  const JoinPlan pl = join_plan(n_fact, n_rows, t, groups, dev);
  if (!partitioned) {
    const size_t lds = join_lds_bytes(groups, t);
    // Every lane's bins must see fewer than 2^19 rows per launch: at most 16
    // waves share a bin, so a thread handles at most 2^14 rows per launch.
    const int64_t per_launch_max = (int64_t)dev.cu_count * kJoinThreads * (1LL << 14);
    if (groups == 16) allow_lds(join_kernel<16>, lds);
    else allow_lds(join_kernel<1>, lds);
    for (int64_t off = 0; off < n_fact; off += per_launch_max) {
      const int64_t n = n_fact - off < per_launch_max ? n_fact - off : per_launch_max;
      const int64_t need = (n + 4LL * kJoinThreads - 1) / (4LL * kJoinThreads);
      const int grid = need < dev.cu_count ? (int)need : dev.cu_count;
      st = stage_begin("join_single_pass", s);
      if (groups == 16)
        hipLaunchKernelGGL(join_kernel<16>, dim3(grid), dim3(kJoinThreads), lds, s, keys + off, n, words, n_rows, t,
                           price, cat, cat_lt, out_sum, out_cnt, flag);
      else
        hipLaunchKernelGGL(join_kernel<1>, dim3(grid), dim3(kJoinThreads), lds, s, keys + off, n, words, n_rows, t,
                           price, cat, cat_lt, out_sum, out_cnt, flag);
      e = hipGetLastError();
      stage_end(st, s);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }

  // Partitioned form, one round of at most pl.round rows at a time.
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

  const size_t lds1 = join_lds_bytes(groups, t_lds) + (size_t)(pl.slices + kWave + 4) * 4;
  const size_t lds3 = (groups == 16 ? (size_t)kJoinBinRows * kWave * 8 : 0) + ((size_t)4 << pl.wshift) +
                      (size_t)(pl.slices + 1) * 4;
  // keys past the last slice (dimensions of more than kMaxSlices slices) are gathered in pass 1
  const int64_t tail_row = (int64_t)t + ((int64_t)pl.slices << pl.wshift);
  const int32_t tail_start = tail_row < n_rows ? (int32_t)tail_row : n_rows;
  const bool gather = tail_start < n_rows || t_lds < t;
  auto split_kernel = groups == 16 ? (gather ? join_split_kernel<16, true> : join_split_kernel<16, false>)
                                   : (gather ? join_split_kernel<1, true> : join_split_kernel<1, false>);
  allow_lds(split_kernel, lds1);
  if (groups == 16) allow_lds(join_slice_kernel<16>, lds3);
  else allow_lds(join_slice_kernel<1>, lds3);
  for (int64_t off = 0; off < n_fact; off += pl.round) {
    const int64_t n = n_fact - off < pl.round ? n_fact - off : pl.round;
    st = stage_begin("join_split", s);
    hipLaunchKernelGGL(split_kernel, dim3(pl.blocks), dim3(kJoinThreads), lds1, s, keys + off, n, words, n_rows,
                       t_lds, t, pl.slices, pl.wshift, tail_start, price, cat, cat_lt, out_sum, out_cnt, flag, seg, pl.seg_cap,
                       tab.seg_count, tab.hist);
    e = hipGetLastError();
    stage_end(st, s);
    st = stage_begin("join_plan", s);
    if (e == hipSuccess) e = launch_partition_plan(tab, pl.slices, pl.blocks, s);
    stage_end(st, s);
    st = stage_begin("join_scatter", s);
    if (e == hipSuccess)
      e = launch_partition_scatter(tab, pl.slices, pl.blocks, seg, nullptr, pl.seg_cap, t, pl.wshift, items, nullptr,
                                   s, t < kCombineBelow);
    stage_end(st, s);
    if (e != hipSuccess) return e;
    st = stage_begin("join_slice", s);
    if (groups == 16)
      hipLaunchKernelGGL(join_slice_kernel<16>, dim3(pl.blocks), dim3(kJoinThreads), lds3, s, items, tab.slice_off,
                         pl.slices, words, n_rows, t, pl.wshift, price, cat, cat_lt, out_sum, out_cnt,
                         flag);
    else
      hipLaunchKernelGGL(join_slice_kernel<1>, dim3(pl.blocks), dim3(kJoinThreads), lds3, s, items, tab.slice_off,
                         pl.slices, words, n_rows, t, pl.wshift, price, cat, cat_lt, out_sum, out_cnt,
                         flag);
    e = hipGetLastError();
    stage_end(st, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace skew

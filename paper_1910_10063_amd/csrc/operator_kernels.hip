// Operator variants of Section 4.1 on the frequency-ordered layout:
// materialization (Q1), selection into compacted fact offsets (Q2) and the
// heavy-hitter counts of Q3a (Section 4.2.2).  All three keep the hot prefix
// of what they consult in LDS, as the join does (Section 4.2).
#include "kernels.h"
#include "profiler.h"
#include "query_common.h"

namespace skew {
namespace {

constexpr int kOpThreads = 1024;
constexpr int kOpWaves = kOpThreads / kWave;
constexpr int kOpVecs = 4;  // 16-byte key vectors per lane per batch

// ---------------------------------------------------------------------------
// Q1 materialization: out[j] = col[keys[j]].  Keys below t read the LDS copy
// of col[0, t); the others gather through a range-checked buffer load, which
// also yields the 0 that a key outside [0, n_rows) materializes.  Workgroup b
// owns a contiguous range of 16-byte vectors (keys and out share their
// alignment); the next batch is loaded while the current one is resolved.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int32_t mat_one(const HotCtx &h, uint32_t n_rows, uint32_t k, bool &bad) {
  bad |= k >= n_rows;
  return (int32_t)fetch_hot_or_global(h, k);
}

__global__ __launch_bounds__(kOpThreads) void materialize_kernel(const int32_t *__restrict__ keys, int64_t n,
                                                                 const int32_t *__restrict__ col, int32_t n_rows,
                                                                 int32_t t, int32_t *__restrict__ out,
                                                                 int32_t *flag) {
  extern __shared__ __align__(16) unsigned char smem[];
  uint32_t *hot = reinterpret_cast<uint32_t *>(smem);
  HotCtx h;
  h.hot = hot;
  h.words = record_buffer(col, (uint32_t)n_rows);
  h.t = (uint32_t)t;
  h.tclamp = t > 0 ? (uint32_t)t - 1 : 0u;
  stage_words(hot, reinterpret_cast<const uint32_t *>(col), 0, t);
  if (t == 0 && threadIdx.x == 0) hot[0] = 0;
  __syncthreads();
  bool bad = false;
  const uint32_t nr = (uint32_t)n_rows;

  if ((((uintptr_t)keys ^ (uintptr_t)out) & 15u) != 0) {  // no common alignment: one row per lane
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride)
      out[j] = mat_one(h, nr, (uint32_t)load_stream1(keys + j), bad);
    if (bad) *flag = 1;
    return;
  }
  const Split4 sp = split4(keys, n);
  {  // scalar head (block 0, lanes 0-2) and tail (last block, lanes 64-66)
    if (blockIdx.x == 0 && threadIdx.x < sp.head) out[threadIdx.x] = mat_one(h, nr, (uint32_t)keys[threadIdx.x], bad);
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x >= kWave && threadIdx.x - kWave < n - sp.tail) {
      const int64_t j = sp.tail + threadIdx.x - kWave;
      out[j] = mat_one(h, nr, (uint32_t)keys[j], bad);
    }
  }
  const i32x4 *vk = reinterpret_cast<const i32x4 *>(keys + sp.head);
  i32x4 *vo = reinterpret_cast<i32x4 *>(out + sp.head);
  const int64_t per = (sp.nvec + gridDim.x - 1) / gridDim.x;
  const int64_t vb = (int64_t)blockIdx.x * per < sp.nvec ? (int64_t)blockIdx.x * per : sp.nvec;
  const int64_t ve = vb + per < sp.nvec ? vb + per : sp.nvec;
  constexpr int64_t kTile = (int64_t)kOpThreads * kOpVecs;
  const int64_t full_end = vb + ((ve - vb) / kTile) * kTile;
  auto resolve = [&](const i32x4(&x)[kOpVecs], int64_t base, bool guard) {
#pragma unroll
    for (int u = 0; u < kOpVecs; ++u) {
      const int64_t vi = base + u * kOpThreads + threadIdx.x;
      if (guard && vi >= ve) continue;
      i32x4 r;
      r.x = mat_one(h, nr, (uint32_t)x[u].x, bad);
      r.y = mat_one(h, nr, (uint32_t)x[u].y, bad);
      r.z = mat_one(h, nr, (uint32_t)x[u].z, bad);
      r.w = mat_one(h, nr, (uint32_t)x[u].w, bad);
      store_stream4(vo + vi, r);
    }
  };
  auto load_tile = [&](i32x4(&x)[kOpVecs], int64_t base) {
#pragma unroll
    for (int u = 0; u < kOpVecs; ++u) x[u] = load_stream4(vk + base + u * kOpThreads + threadIdx.x);
  };
  i32x4 xa[kOpVecs], xb[kOpVecs];
  int64_t base = vb;
  if (base < full_end) load_tile(xa, base);
  while (base < full_end) {  // unconditional prefetch: the last one re-reads the current tile
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
    i32x4 x[kOpVecs];
#pragma unroll
    for (int u = 0; u < kOpVecs; ++u) {
      const int64_t vi = full_end + u * kOpThreads + threadIdx.x;
      x[u] = vi < ve ? load_stream4(vk + vi) : i32x4{0, 0, 0, 0};
    }
    resolve(x, full_end, true);
  }
  if (bad) *flag = 1;
}

// ---------------------------------------------------------------------------
// Q2 selection.  The predicate is evaluated once per dimension row into a
// bitmap (bit r of word r / 32), as in Section 4.1; rows below t (bits) are
// tested against an LDS copy of the bitmap's first words.  Every wave owns a
// contiguous chunk of fact rows and appends the offsets of its qualifying
// rows, in row order, to its own segment (ballots + lane counts, the GPU form
// of a compressed store); a scan of the segment counts and a copy concatenate
// the segments.
// ---------------------------------------------------------------------------
__global__ void select_pack_kernel(const int32_t *__restrict__ col, int32_t n_rows, int32_t lt,
                                   uint32_t *__restrict__ bitmap, int32_t *flag, int64_t *count) {
  const int64_t nchunks = ((int64_t)n_rows + kWave - 1) / kWave;  // 64 rows -> 2 bitmap words
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nwaves = (int64_t)gridDim.x * blockDim.x / kWave;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *flag = 0;
    *count = 0;
  }
  const int64_t nwords = ((int64_t)n_rows + 31) / 32;
  for (int64_t c = wave; c < nchunks; c += nwaves) {
    const int64_t r = c * kWave + lane_id();
    const bool q = r < n_rows && col[r] < lt;
    const uint64_t m = __ballot(q);
    if (lane_id() == 0) bitmap[2 * c] = (uint32_t)m;
    if (lane_id() == 1 && 2 * c + 1 < nwords) bitmap[2 * c + 1] = (uint32_t)(m >> 32);
  }
}

struct BitCtx {
  const uint32_t *hot;  // LDS: bitmap words [0, hot_words)
  rsrc_t words;         // bitmap in global memory, range-checked
  uint32_t t;           // rows [0, t) are tested in LDS
  uint32_t wclamp;      // last LDS word
  uint32_t n_rows;
};

// Bit of row k: a clamped LDS read and a buffer gather pushed out of range for
// hot rows (no memory traffic), the select keeps the right word.
__device__ __forceinline__ bool test_bit(const BitCtx &b, uint32_t k, bool &bad) {
  bad |= k >= b.n_rows;
  const bool hot = k < b.t;
  const uint32_t wi = k >> 5;
  const uint32_t wl = b.hot[wi < b.wclamp ? wi : b.wclamp];
  const uint32_t wg = buffer_load_record(b.words, (int32_t)(hot ? 0xFFFFFFFFu : wi), 0, 0, 0);
  return (((hot ? wl : wg) >> (k & 31u)) & 1u) != 0;
}

// Rows of the wave chunk s: vectors [s * cv, min((s + 1) * cv, nvec)) when the
// keys are 16-byte aligned (rows 4 nvec .. n - 1 form one more chunk, S),
// else rows [s * cv, min((s + 1) * cv, n)).  Segment s starts at s * cap.
struct SelectPlan {
  int64_t n;       // rows of this round
  int64_t nvec;    // 16-byte vectors (aligned case), 0 otherwise
  int64_t cv;      // vectors (or rows) per chunk
  int64_t cap;     // segment slots per chunk
  int32_t chunks;  // S (+ 1 for the tail chunk)
  int32_t aligned; // keys start 16-byte aligned
};

__global__ __launch_bounds__(kOpThreads) void select_kernel(const int32_t *__restrict__ keys, SelectPlan pl,
                                                            const uint32_t *__restrict__ bitmap, int32_t n_rows,
                                                            int32_t t, int32_t row_base, int32_t *__restrict__ seg,
                                                            uint32_t *__restrict__ seg_count, int32_t *flag) {
  extern __shared__ __align__(16) unsigned char smem[];
  uint32_t *hot = reinterpret_cast<uint32_t *>(smem);
  const int32_t hot_words = (int32_t)(((int64_t)t + 31) / 32);
  stage_words(hot, bitmap, 0, hot_words);
  if (hot_words == 0 && threadIdx.x == 0) hot[0] = 0;
  __syncthreads();
  BitCtx b;
  b.hot = hot;
  b.words = record_buffer(bitmap, (uint32_t)(((int64_t)n_rows + 31) / 32));
  b.t = (uint32_t)t;
  b.wclamp = hot_words > 0 ? (uint32_t)hot_words - 1 : 0u;
  b.n_rows = (uint32_t)n_rows;
  bool bad = false;

  const int64_t s = (int64_t)blockIdx.x * kOpWaves + threadIdx.x / kWave;  // this wave's chunk
  if (s >= pl.chunks) return;
  const rsrc_t out = record_buffer(seg + s * pl.cap, (uint32_t)pl.cap);
  uint32_t running = 0;
  if (pl.aligned) {
    // aligned: chunk s < S covers vectors, chunk S the last n - 4 nvec rows
    const int64_t S = pl.chunks - 1;
    if (s < S) {
      const i32x4 *vk = reinterpret_cast<const i32x4 *>(keys);
      const int64_t v0 = s * pl.cv;
      const int64_t v1 = v0 + pl.cv < pl.nvec ? v0 + pl.cv : pl.nvec;
      for (int64_t vb = v0; vb < v1; vb += (int64_t)kWave * kOpVecs) {
        i32x4 x[kOpVecs];
#pragma unroll
        for (int u = 0; u < kOpVecs; ++u) {
          const int64_t vi = vb + u * kWave + lane_id();
          x[u] = vi < v1 ? load_stream4(vk + vi) : i32x4{0, 0, 0, 0};
        }
#pragma unroll
        for (int u = 0; u < kOpVecs; ++u) {
          const int64_t vi = vb + u * kWave + lane_id();
          const bool ok = vi < v1;
          const uint32_t k4[4] = {(uint32_t)x[u].x, (uint32_t)x[u].y, (uint32_t)x[u].z, (uint32_t)x[u].w};
          bool sel[4];
          uint64_t m[4];
          uint32_t below = 0, total = 0;
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            sel[j] = ok && test_bit(b, k4[j], bad);
            m[j] = __ballot(sel[j]);
            below += __builtin_amdgcn_mbcnt_hi((uint32_t)(m[j] >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m[j], 0u));
            total += (uint32_t)__popcll(m[j]);
          }
          uint32_t pos = running + below;
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            buffer_store_record(row_base + (int32_t)(4 * vi + j), out, sel[j] ? (int32_t)pos : -1, 0, 0, 0);
            pos += sel[j] ? 1u : 0u;
          }
          running += total;
        }
      }
    } else {  // tail rows 4 nvec .. n - 1 (at most 3)
      const int64_t j = 4 * pl.nvec + lane_id();
      const bool sel = j < pl.n && test_bit(b, (uint32_t)keys[j], bad);
      const uint64_t m = __ballot(sel);
      buffer_store_record(row_base + (int32_t)j, out,
                          sel ? (int32_t)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                   __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u))
                              : -1,
                          0, 0, 0);
      running = (uint32_t)__popcll(m);
    }
  } else {  // unaligned keys: one row per lane, chunk s covers rows [s cv, (s + 1) cv)
    const int64_t r0 = s * pl.cv;
    const int64_t r1 = r0 + pl.cv < pl.n ? r0 + pl.cv : pl.n;
    for (int64_t rb = r0; rb < r1; rb += kWave) {
      const int64_t j = rb + lane_id();
      const bool sel = j < r1 && test_bit(b, (uint32_t)load_stream1(keys + j), bad);
      const uint64_t m = __ballot(sel);
      const uint32_t pos =
          running + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
      buffer_store_record(row_base + (int32_t)j, out, sel ? (int32_t)pos : -1, 0, 0, 0);
      running += (uint32_t)__popcll(m);
    }
  }
  if (lane_id() == 0) seg_count[s] = running;
  if (bad) *flag = 1;
}

// Block s copies segment s to out[*count + off[s] ...]; the round total is
// added to *count by select_advance_kernel afterwards.
__global__ void select_copy_kernel(const int32_t *__restrict__ seg, int64_t cap, const uint32_t *__restrict__ seg_count,
                                   const uint32_t *__restrict__ seg_off, const int64_t *__restrict__ count,
                                   int32_t *__restrict__ out) {
  const int64_t s = blockIdx.x;
  const uint32_t c = seg_count[s];
  int32_t *dst = out + *count + seg_off[s];
  const int32_t *src = seg + s * cap;
  for (uint32_t i = threadIdx.x; i < c; i += blockDim.x) dst[i] = src[i];
}

__global__ void select_advance_kernel(int64_t *count, const uint32_t *round_total) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *count += *round_total;
}

// ---------------------------------------------------------------------------
// Q3a heavy hitters (Section 4.2.2): counts of the ranks below k on the
// frequency-ordered layout; every other row is dropped.  Ranks below 16 have
// one counter per wave lane, ranks below kc one counter per workgroup in LDS,
// ranks in [kc, k) go to global atomics.
// ---------------------------------------------------------------------------
constexpr int kHeavyCopies = 16;
constexpr int kHeavyCopySlots = kHeavyCopies * kWave;

struct HeavyCtx {
  uint32_t *cnt;  // LDS: [kHeavyCopySlots] copies | [kc] bins | [64] sink
  uint32_t k, kc, ncopy, n_keys;
  uint64_t *out;
  bool bad;
};

__device__ __forceinline__ void heavy_one(HeavyCtx &c, uint32_t g) {
  c.bad |= g >= c.n_keys;
  const uint32_t sink = kHeavyCopySlots + c.kc + lane_id();
  const uint32_t i = g < c.ncopy ? g * kWave + lane_id() : (g < c.kc ? kHeavyCopySlots + g : sink);
  lds_add_u32(&c.cnt[i], 1u);
  if (__builtin_expect(g >= c.kc && g < c.k, 0)) global_add_u64(&c.out[g], 1ull);
}

__global__ void heavy_prep_kernel(const int32_t *__restrict__ perm, int32_t k, int32_t *__restrict__ out_keys,
                                  int64_t *__restrict__ out_count, int32_t *flag) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid == 0) *flag = 0;
  for (int64_t r = gid; r < k; r += (int64_t)gridDim.x * blockDim.x) {
    out_keys[r] = perm ? perm[r] : (int32_t)r;
    out_count[r] = 0;
  }
}

__global__ __launch_bounds__(kOpThreads) void heavy_kernel(const int32_t *__restrict__ keys, int64_t n, int32_t k,
                                                           int32_t kc, int32_t n_keys, int64_t *__restrict__ out,
                                                           int32_t *flag) {
  extern __shared__ __align__(16) unsigned char smem[];
  HeavyCtx c;
  c.cnt = reinterpret_cast<uint32_t *>(smem);
  c.k = (uint32_t)k;
  c.kc = (uint32_t)kc;
  c.ncopy = kc < kHeavyCopies ? (uint32_t)kc : (uint32_t)kHeavyCopies;
  c.n_keys = (uint32_t)n_keys;
  c.out = reinterpret_cast<uint64_t *>(out);
  c.bad = false;
  for (int i = threadIdx.x; i < kHeavyCopySlots + kc + kWave; i += blockDim.x) c.cnt[i] = 0;
  __syncthreads();
  const Split4 sp = split4(keys, n);
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t T = (int64_t)gridDim.x * blockDim.x;
  if (gid < sp.head) heavy_one(c, (uint32_t)keys[gid]);
  if (gid < n - sp.tail) heavy_one(c, (uint32_t)keys[sp.tail + gid]);
  const i32x4 *vk = reinterpret_cast<const i32x4 *>(keys + sp.head);
  int64_t v = gid;
  for (; v + (kOpVecs - 1) * T < sp.nvec; v += kOpVecs * T) {
    i32x4 x[kOpVecs];
#pragma unroll
    for (int u = 0; u < kOpVecs; ++u) x[u] = load_stream4(vk + v + u * T);
#pragma unroll
    for (int u = 0; u < kOpVecs; ++u) {
      heavy_one(c, (uint32_t)x[u].x);
      heavy_one(c, (uint32_t)x[u].y);
      heavy_one(c, (uint32_t)x[u].z);
      heavy_one(c, (uint32_t)x[u].w);
    }
  }
  for (; v < sp.nvec; v += T) {
    const i32x4 x = load_stream4(vk + v);
    heavy_one(c, (uint32_t)x.x);
    heavy_one(c, (uint32_t)x.y);
    heavy_one(c, (uint32_t)x.z);
    heavy_one(c, (uint32_t)x.w);
  }
  if (c.bad) *flag = 1;
  __syncthreads();
  const int w = threadIdx.x / kWave;
  for (uint32_t g = w; g < c.ncopy; g += kOpWaves) {
    const uint64_t s = wave_sum_u64((uint64_t)c.cnt[g * kWave + lane_id()]);
    if (lane_id() == 0 && s) global_add_u64(&c.out[g], s);
  }
  for (uint32_t g = c.ncopy + threadIdx.x; g < c.kc; g += blockDim.x) {
    const uint32_t s = c.cnt[kHeavyCopySlots + g];
    if (s) global_add_u64(&c.out[g], (uint64_t)s);
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

constexpr size_t kStaticReserve = 1024;  // LDS kept free for the compiler's own use

}  // namespace

// ---------------------------------------------------------------------------
// Capacities and launchers
// ---------------------------------------------------------------------------
int32_t materialize_max_hot_rows(const DeviceInfo &dev) {
  if (dev.lds_per_block <= kStaticReserve + 16) return 0;
  return (int32_t)(((dev.lds_per_block - kStaticReserve) / 4) & ~(size_t)3);
}

int64_t select_max_hot_rows(const DeviceInfo &dev) {
  if (dev.lds_per_block <= kStaticReserve + 16) return 0;
  return (int64_t)(((dev.lds_per_block - kStaticReserve) / 4) & ~(size_t)3) * 32;
}

int32_t heavy_max_lds_ranks(const DeviceInfo &dev) {
  const size_t fixed = (size_t)(kHeavyCopySlots + kWave) * 4 + kStaticReserve;
  if (dev.lds_per_block <= fixed) return 0;
  return (int32_t)((dev.lds_per_block - fixed) / 4);
}

hipError_t launch_materialize(const int32_t *keys, int64_t n, const int32_t *col, int32_t n_rows, int32_t t,
                              int32_t *out, int32_t *flag, const DeviceInfo &dev, hipStream_t s) {
  const int32_t cap = materialize_max_hot_rows(dev);
  if (t > cap) t = cap;
  if (t > n_rows) t = n_rows;
  if (t < 0) t = 0;
  StageTimer st = stage_begin("materialize_flag", s);
  hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t *>(flag), 1, 0u, s);
  stage_end(st, s);
  if (e != hipSuccess || n == 0) return e;
  const size_t lds = (size_t)((t + 4) & ~3) * 4;
  allow_lds(materialize_kernel, lds);
  const int64_t need = (n + 4LL * kOpThreads * kOpVecs - 1) / (4LL * kOpThreads * kOpVecs);
  const int grid = need < dev.cu_count ? (int)need : dev.cu_count;
  st = stage_begin("materialize", s);
  hipLaunchKernelGGL(materialize_kernel, dim3(grid > 0 ? grid : 1), dim3(kOpThreads), lds, s, keys, n, col, n_rows,
                     t, out, flag);
  e = hipGetLastError();
  stage_end(st, s);
  return e;
}

size_t select_round_rows() { return (size_t)1 << 28; }

// Segment slots of one round of `round` rows over S wave chunks: at most
// (S + 1) chunks of 4 ceil(ceil(round / 4) / S) slots (16-byte aligned keys),
// or S chunks of ceil(round / S) slots.
size_t select_seg_slots(int64_t round, int32_t S) { return (size_t)round + (size_t)round / S + 4 * (size_t)S + 8; }

size_t select_workspace_bytes(int64_t n_fact, int32_t n_rows, int32_t blocks) {
  auto r = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const int64_t round = n_fact < (int64_t)select_round_rows() ? n_fact : (int64_t)select_round_rows();
  const int32_t S = blocks * kOpWaves;
  return r(((size_t)n_rows + 31) / 32 * 4 + 8)      // bitmap
         + r(select_seg_slots(round, S) * 4)         // segments
         + 2 * r((size_t)(S + 2) * 4) + r(4);        // counts, offsets, round total
}

hipError_t launch_select(const int32_t *keys, int64_t n_fact, const int32_t *col, int32_t n_rows, int32_t lt,
                         int32_t t, int32_t *out, int64_t *count, int32_t *flag, void *ws, const DeviceInfo &dev,
                         hipStream_t s) {
  auto r = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const int blocks = dev.cu_count > 0 ? dev.cu_count : 256;
  const int32_t S = blocks * kOpWaves;
  char *w = (char *)ws;
  uint32_t *bitmap = (uint32_t *)w;
  w += r(((size_t)n_rows + 31) / 32 * 4 + 8);
  const int64_t round = n_fact < (int64_t)select_round_rows() ? n_fact : (int64_t)select_round_rows();
  int32_t *seg = (int32_t *)w;
  w += r(select_seg_slots(round, S) * 4);
  uint32_t *seg_count = (uint32_t *)w;
  w += r((size_t)(S + 2) * 4);
  uint32_t *seg_off = (uint32_t *)w;
  w += r((size_t)(S + 2) * 4);
  uint32_t *round_total = (uint32_t *)w;

  const int64_t cap_bits = select_max_hot_rows(dev);
  int64_t tt = t;
  if (tt > cap_bits) tt = cap_bits;
  if (tt > n_rows) tt = n_rows;
  if (tt < 0) tt = 0;
  StageTimer st = stage_begin("select_pack", s);
  const int64_t nchunks = ((int64_t)n_rows + kWave - 1) / kWave;
  hipLaunchKernelGGL(select_pack_kernel, dim3(grid_1d(nchunks * kWave, 256, dev.cu_count * 8)), dim3(256), 0, s, col,
                     n_rows, lt, bitmap, flag, count);
  hipError_t e = hipGetLastError();
  stage_end(st, s);
  if (e != hipSuccess || n_fact == 0) return e;
  const size_t lds = (size_t)(((tt + 31) / 32 + 4) & ~3) * 4;
  allow_lds(select_kernel, lds);
  for (int64_t off = 0; off < n_fact; off += round) {
    const int64_t n = n_fact - off < round ? n_fact - off : round;
    const int32_t *k = keys + off;
    SelectPlan pl;
    pl.n = n;
    pl.aligned = ((uintptr_t)k & 15u) == 0;
    if (pl.aligned) {
      pl.nvec = n / 4;
      pl.cv = (pl.nvec + S - 1) / S;
      if (pl.cv < 1) pl.cv = 1;
      pl.cap = 4 * pl.cv;
      pl.chunks = S + 1;  // + the tail chunk
    } else {
      pl.nvec = 0;
      pl.cv = (n + S - 1) / S;
      if (pl.cv < 1) pl.cv = 1;
      pl.cap = pl.cv;
      pl.chunks = S;
    }
    st = stage_begin("select", s);
    hipLaunchKernelGGL(select_kernel, dim3((pl.chunks + kOpWaves - 1) / kOpWaves), dim3(kOpThreads), lds, s, k, pl,
                       bitmap, n_rows, (int32_t)tt, (int32_t)off, seg, seg_count, flag);
    e = hipGetLastError();
    stage_end(st, s);
    st = stage_begin("select_scan", s);
    if (e == hipSuccess) e = hipMemcpyAsync(seg_off, seg_count, (size_t)pl.chunks * 4, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = launch_exclusive_scan(seg_off, pl.chunks, round_total, nullptr, s);
    stage_end(st, s);
    st = stage_begin("select_copy", s);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(select_copy_kernel, dim3(pl.chunks), dim3(256), 0, s, seg, pl.cap, seg_count, seg_off, count,
                         out);
      e = hipGetLastError();
    }
    if (e == hipSuccess) {
      hipLaunchKernelGGL(select_advance_kernel, dim3(1), dim3(64), 0, s, count, round_total);
      e = hipGetLastError();
    }
    stage_end(st, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_heavy(const int32_t *keys, int64_t n_fact, int32_t n_keys, int32_t k, const int32_t *perm,
                        int32_t *out_keys, int64_t *out_count, int32_t *flag, const DeviceInfo &dev, hipStream_t s) {
  StageTimer st = stage_begin("heavy_prep", s);
  hipLaunchKernelGGL(heavy_prep_kernel, dim3(grid_1d(k > 0 ? k : 1, 256, dev.cu_count * 16)), dim3(256), 0, s, perm, k,
                     out_keys,
                     out_count, flag);
  hipError_t e = hipGetLastError();
  stage_end(st, s);
  if (e != hipSuccess || n_fact == 0 || k == 0) return e;
  const int32_t cap = heavy_max_lds_ranks(dev);
  const int32_t kc = k < cap ? k : cap;
  const size_t lds = (size_t)(kHeavyCopySlots + kc + kWave) * 4;
  allow_lds(heavy_kernel, lds);
  // LDS counters are 32-bit: at most 2^31 rows per workgroup and launch.
  const int64_t per_launch_max = (int64_t)dev.cu_count * (1LL << 31);
  for (int64_t off = 0; off < n_fact; off += per_launch_max) {
    const int64_t n = n_fact - off < per_launch_max ? n_fact - off : per_launch_max;
    const int64_t need = (n + 4LL * kOpThreads - 1) / (4LL * kOpThreads);
    const int grid = need < dev.cu_count ? (int)need : dev.cu_count;
    st = stage_begin("heavy", s);
    hipLaunchKernelGGL(heavy_kernel, dim3(grid > 0 ? grid : 1), dim3(kOpThreads), lds, s, keys + off, n, k, kc,
                       n_keys, out_count, flag);
    e = hipGetLastError();
    stage_end(st, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace skew

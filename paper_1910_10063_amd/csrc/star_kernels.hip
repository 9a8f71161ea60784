// Batched star join: many fact tables of uneven sizes, each joined with a
// product dimension (price summed by category) and a customer dimension that
// filters (segment < threshold of the query), all in one persistent kernel.
// Workgroups take tiles of rows from a device work queue; a tile never spans
// two queries.  Both dimensions keep their hot prefix in LDS (Section 4.2:
// on the frequency-ordered layouts the hot rows are the first ones) and the
// rest is gathered through range-checked buffer loads.  The product prefix is
// one packed word per row, shared by all queries.  The customer prefix is the
// filter's outcome, one bit per row, so a workgroup holds eight times more
// hot customers than it would segments; every query has its own bitmap,
// built before the batch kernel and staged into LDS when a workgroup moves on
// to a tile of another query.  When the bitmaps of all queries over every
// customer row fit a fixed budget, they are built for every row, and a cold
// customer row reads its bit from the query's bitmap in global memory (a
// 2e6-row dimension is 250 KB of bits per query, against 2 MB of segments
// shared by all queries, so the rows the queries read stay in L2 next to
// more of the product words).  Every launch here is a kernel (no memset or
// host copy), so the whole call can be captured in a HIP graph and replayed.
#include "kernels.h"
#include "profiler.h"
#include "query_common.h"

namespace skew {
namespace {

constexpr int kStarThreads = 1024;
constexpr int kStarVecs = 2;       // 16-byte vectors of each key column per lane per batch
// Bins 1..16 are the groups and bin 0 the sink: every word the kernel adds is
// a packed product word (group field category + 1 <= 16), kValid (field 0) or
// 0, so the 5-bit group field never exceeds 16.
constexpr int kStarBins = 17;
constexpr int kBitsThreads = 256;
constexpr int kBitsQueries = 8;    // queries per workgroup of the bitmap kernel

// Product word: kValid | (category + 1) << 25 | price, kValid alone for a row
// outside every group, 0 when the price does not fit (slow path).
__global__ void star_pack_kernel(const int32_t *__restrict__ price, const int8_t *__restrict__ cat, int32_t n_prod,
                                 uint32_t *__restrict__ words, const int8_t *__restrict__ attr, int32_t n_cust,
                                 int8_t *__restrict__ attr_copy, int32_t attr_padded) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = gid; r < n_prod; r += stride) {
    const int32_t p = price[r];
    const int32_t c = cat[r];
    uint32_t w = kValid;
    if (c >= 0 && c < 16) w = ((uint32_t)p <= kPriceMask) ? (kValid | ((uint32_t)(c + 1) << kGroupShift) | (uint32_t)p) : 0u;
    words[r] = w;
  }
  // customer segments, padded to whole 32-row groups (the padding rows are
  // past the dimension and never pass: every lookup checks the row first)
  for (int64_t r = gid; r < attr_padded; r += stride) attr_copy[r] = r < n_cust ? attr[r] : (int8_t)127;
}

// Customer bitmaps of the hot prefix: bit u of query q's bitmap (word u / 32,
// bit u % 32) is set when segment[u] < threshold[q], for rows [0, tc).  One
// thread reads the 32 segments of one word once and writes that word for
// kBitsQueries queries; the bitmaps are `stride` words apart.
__global__ __launch_bounds__(kBitsThreads) void star_bits_kernel(const uint4 *__restrict__ segs, int32_t n_words,
                                                                 const int32_t *__restrict__ qlt, int32_t nq,
                                                                 int32_t stride, uint32_t *__restrict__ bits) {
  const int32_t w = blockIdx.x * kBitsThreads + threadIdx.x;
  if (w >= n_words) return;
  const uint4 a = segs[2 * w], b = segs[2 * w + 1];  // rows 32w .. 32w + 31
  const uint32_t sw[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
  const int32_t q0 = blockIdx.y * kBitsQueries;
  const int32_t q1 = q0 + kBitsQueries < nq ? q0 + kBitsQueries : nq;
  for (int32_t q = q0; q < q1; ++q) {
    const int32_t lt = qlt[q];
    uint32_t word = 0;
#pragma unroll
    for (int i = 0; i < 32; ++i) word |= (uint32_t)((int32_t)(int8_t)(sw[i >> 2] >> (8 * (i & 3))) < lt) << i;
    bits[(int64_t)q * stride + w] = word;
  }
}

__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t x) {
  const int lane = lane_id();
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, kWave);
    if (lane >= o) x += y;
  }
  return x;
}

// Tile table: tiles of query q start at tile_start[q]; outputs and the queue
// counter are cleared (one workgroup, n_queries <= kMaxStarQueries).
__global__ __launch_bounds__(1024) void star_plan_kernel(const int64_t *__restrict__ qstart, int32_t nq,
                                                         int64_t tile_rows, uint32_t *__restrict__ tile_start,
                                                         uint32_t *__restrict__ counter, int64_t *__restrict__ out_sum,
                                                         int64_t *__restrict__ out_cnt, int32_t *flag) {
  __shared__ uint32_t part[64];  // [0, 16): wave totals, [32, 48): their exclusive prefixes
  for (int i = threadIdx.x; i < nq * 16; i += blockDim.x) {
    out_sum[i] = 0;
    out_cnt[i] = 0;
  }
  if (threadIdx.x == 0) {
    *counter = 0;
    *flag = 0;
  }
  // tile counts of this thread's queries (ceil(nq / 1024) consecutive ones)
  const int per = (nq + 1023) / 1024;
  const int q0 = threadIdx.x * per;
  uint32_t sum = 0;
  for (int q = q0; q < q0 + per && q < nq; ++q) {
    const int64_t n = qstart[q + 1] - qstart[q];
    sum += n > 0 ? (uint32_t)((n + tile_rows - 1) / tile_rows) : 0u;
  }
  // exclusive scan over the 1024 threads: within each wave, then over the 16 wave totals
  const uint32_t incl = wave_inclusive_scan(sum);
  if (lane_id() == kWave - 1) part[threadIdx.x / kWave] = incl;
  __syncthreads();
  if (threadIdx.x < kWave) {
    const uint32_t w = threadIdx.x < 1024 / kWave ? part[threadIdx.x] : 0u;
    const uint32_t wi = wave_inclusive_scan(w);
    if (threadIdx.x < 1024 / kWave) part[32 + threadIdx.x] = wi - w;
    if (threadIdx.x == 1024 / kWave - 1) tile_start[nq] = wi;
  }
  __syncthreads();
  uint32_t run = part[32 + threadIdx.x / kWave] + incl - sum;
  for (int q = q0; q < q0 + per && q < nq; ++q) {
    tile_start[q] = run;
    const int64_t n = qstart[q + 1] - qstart[q];
    run += n > 0 ? (uint32_t)((n + tile_rows - 1) / tile_rows) : 0u;
  }
}

struct StarCtx {
  const uint32_t *phot;  // LDS: product words [0, tp)
  uint32_t tp, tpclamp;
  rsrc_t pwords;         // all product words (range-checked)
  const uint32_t *chot;  // LDS: the current query's customer bitmap, rows [0, tc)
  uint32_t tc, tcclamp;  // tc in rows (bits), tcclamp in words
  rsrc_t cwords;         // all customer segments, four to a word (range-checked)
  rsrc_t cbits;          // FULL: the current query's bitmap over every customer row (range-checked)
  uint32_t n_prod, n_cust;
};

// Whether customer row u < n_cust passes the query's filter: a bit of the
// LDS bitmap for a hot row; for a cold one, its bit of the query's bitmap in
// global memory (FULL) or its segment, gathered and compared.  The gather
// index is pushed out of range for hot rows, so they cost no memory traffic.
template <bool FULL>
__device__ __forceinline__ bool cust_pass(const StarCtx &x, uint32_t u, int32_t lt) {
  const bool hot = u < x.tc;
  const uint32_t wi = u >> 5;
  const uint32_t bl = x.chot[wi < x.tcclamp ? wi : x.tcclamp] >> (u & 31u);
  if (FULL) {
    const uint32_t wg = buffer_load_record(x.cbits, (int32_t)(hot ? 0xFFFFFFFFu : wi), 0, 0, 0);
    return ((hot ? bl : wg >> (u & 31u)) & 1u) != 0u;
  }
  const uint32_t wg = buffer_load_record(x.cwords, (int32_t)(hot ? 0xFFFFFFFFu : (u >> 2)), 0, 0, 0);
  const int32_t seg = (int32_t)(int8_t)(wg >> (8 * (u & 3u)));
  return hot ? (bl & 1u) != 0u : seg < lt;
}

// Product word of row p for a row whose customer passed; for the other rows
// the gather index is pushed out of range, so a filtered row costs no memory
// traffic (their word is never used).
__device__ __forceinline__ uint32_t prod_word(const StarCtx &x, uint32_t p, bool pass) {
  const bool hot = p < x.tp;
  const uint32_t wl = x.phot[p < x.tpclamp ? p : x.tpclamp];
  const uint32_t wg = buffer_load_record(x.pwords, (int32_t)(hot || !pass ? 0xFFFFFFFFu : p), 0, 0, 0);
  return hot ? wl : wg;
}

struct StarAcc {
  uint64_t *bins;  // LDS [kStarBins][64]: count << 44 | sum, bin 0 a sink
  const int32_t *price;
  const int8_t *cat;
  int64_t *out_sum, *out_cnt;  // this query's 16 groups
  bool bad;
};

__device__ __forceinline__ void star_add(StarAcc &a, uint32_t w) {
  const uint32_t bin = (w >> kGroupShift) & (kJoinBins - 1);
  lds_add_u64(&a.bins[bin * kWave + lane_id()], (1ull << kCountShift) | (w & kPriceMask));
}

// Rare path: a key outside its dimension (joins nothing, sets the flag), or a
// qualifying product row whose price does not fit the word.
__device__ __forceinline__ void star_slow(StarAcc &a, const StarCtx &x, uint32_t p, uint32_t u) {
  if (p >= x.n_prod || u >= x.n_cust) {
    a.bad = true;
    return;
  }
  const int32_t g = a.cat[p];
  if (g < 0 || g >= 16) return;
  global_add_u64(reinterpret_cast<uint64_t *>(&a.out_sum[g]), (uint64_t)(int64_t)a.price[p]);
  global_add_u64(reinterpret_cast<uint64_t *>(&a.out_cnt[g]), 1ull);
}

// One row: product word if the customer passes, the sink bin otherwise.
template <bool FULL>
__device__ __forceinline__ void star_row(StarAcc &a, const StarCtx &x, uint32_t p, uint32_t u, int32_t lt) {
  const bool pass = u < x.n_cust && cust_pass<FULL>(x, u, lt);
  const uint32_t wp = prod_word(x, p, pass);
  const uint32_t w = pass ? wp : kValid;
  star_add(a, w);
  if (__builtin_expect((pass && wp == 0u) || p >= x.n_prod || u >= x.n_cust, 0)) star_slow(a, x, p, u);
}

struct KeyPair {
  i32x4 p, u;
};

// Flush the bins of the current query: 16 waves, wave g sums bin g + 1.
__device__ __forceinline__ void star_flush(StarAcc &a) {
  __syncthreads();
  const int g = threadIdx.x / kWave;
  if (g < 16) {
    uint64_t *b = &a.bins[(g + 1) * kWave + lane_id()];
    const uint64_t e = *b;
    *b = 0;
    const uint64_t s = wave_sum_u64(e & kSumMask);
    const uint64_t k = wave_sum_u64(e >> kCountShift);
    if (lane_id() == 0 && k) {
      global_add_u64(reinterpret_cast<uint64_t *>(&a.out_sum[g]), s);
      global_add_u64(reinterpret_cast<uint64_t *>(&a.out_cnt[g]), k);
    }
  }
  __syncthreads();
}

template <bool FULL>
__global__ __launch_bounds__(kStarThreads) void star_batch_kernel(
    const int32_t *__restrict__ pkeys, const int32_t *__restrict__ ukeys, const int64_t *__restrict__ qstart,
    const int32_t *__restrict__ qlt, int32_t nq, const uint32_t *__restrict__ tile_start, uint32_t *counter,
    int64_t tile_rows, const uint32_t *__restrict__ pwords, int32_t n_prod, int32_t tp,
    const uint32_t *__restrict__ cwords, int32_t n_cust, int32_t tc, const int32_t *__restrict__ price,
    const int8_t *__restrict__ cat, const uint32_t *__restrict__ cbits, int32_t cstride,
    int64_t *__restrict__ out_sum, int64_t *__restrict__ out_cnt, int32_t *flag) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ uint32_t s_tile;
  uint64_t *bins = reinterpret_cast<uint64_t *>(smem);
  uint32_t *phot = reinterpret_cast<uint32_t *>(smem + kStarBins * kWave * 8);
  const int32_t tp_words = (tp + 4) & ~3;
  uint32_t *chot = phot + tp_words;
  const int32_t tc_bits_words = (tc + 31) / 32;
  uint32_t *lts = chot + ((tc_bits_words + 4) & ~3);  // [nq + 1] tile starts
  for (int i = threadIdx.x; i < kStarBins * kWave; i += blockDim.x) bins[i] = 0;
  stage_words(phot, pwords, 0, tp);
  if (tp == 0 && threadIdx.x == 0) phot[0] = 0;
  if (threadIdx.x == 0) chot[0] = 0;  // read (clamped) when tc == 0
  for (int q = threadIdx.x; q <= nq; q += blockDim.x) lts[q] = tile_start[q];
  __syncthreads();

  StarCtx x;
  x.phot = phot;
  x.tp = (uint32_t)tp;
  x.tpclamp = tp > 0 ? (uint32_t)tp - 1 : 0u;
  x.pwords = record_buffer(pwords, (uint32_t)n_prod);
  x.chot = chot;
  x.tc = (uint32_t)tc;
  x.tcclamp = tc > 0 ? (uint32_t)tc_bits_words - 1 : 0u;
  x.cwords = record_buffer(cwords, (uint32_t)((n_cust + 3) / 4));
  x.n_prod = (uint32_t)n_prod;
  x.n_cust = (uint32_t)n_cust;
  StarAcc a;
  a.bins = bins;
  a.price = price;
  a.cat = cat;
  a.bad = false;
  const uint32_t total = lts[nq];
  const i32x4 *vp = reinterpret_cast<const i32x4 *>(pkeys);
  const i32x4 *vu = reinterpret_cast<const i32x4 *>(ukeys);
  int32_t staged_q = -1;  // query whose bitmap is in LDS

  for (;;) {
    if (threadIdx.x == 0) s_tile = atomicAdd(counter, 1u);
    __syncthreads();
    const uint32_t tile = s_tile;
    __syncthreads();  // every thread has read s_tile before it is written again
    if (tile >= total) break;
    int32_t lo_q = 0, hi_q = nq - 1;  // last query whose first tile is <= tile
    while (lo_q < hi_q) {
      const int32_t m = (lo_q + hi_q + 1) >> 1;
      if (lts[m] <= tile) lo_q = m;
      else hi_q = m - 1;
    }
    const int32_t q = lo_q;
    if (q != staged_q && tc > 0) {  // uniform: every thread has the same tile; the last tile's reads are done
      stage_words(chot, cbits, (int64_t)q * cstride, tc_bits_words);
      __syncthreads();
    }
    if (FULL) x.cbits = record_buffer(cbits + (int64_t)q * cstride, (uint32_t)(((int64_t)n_cust + 31) / 32));
    staged_q = q;
    const int64_t r0 = qstart[q] + (int64_t)(tile - lts[q]) * tile_rows;
    const int64_t r1 = r0 + tile_rows < qstart[q + 1] ? r0 + tile_rows : qstart[q + 1];
    const int32_t lt = qlt[q];
    a.out_sum = out_sum + (int64_t)q * 16;
    a.out_cnt = out_cnt + (int64_t)q * 16;
    // rows [r0, r1) as item offsets from r0's 16-byte block
    const int64_t base = r0 & ~(int64_t)3;
    const i32x4 *bp = vp + base / 4;
    const i32x4 *bu = vu + base / 4;
    const int32_t *sp = pkeys + base;
    const int32_t *su = ukeys + base;
    walk_items<4, kStarVecs, kStarThreads, KeyPair>(
        (uint32_t)(r0 - base), (uint32_t)(r1 - base),
        [&](uint32_t i) { star_row<FULL>(a, x, (uint32_t)sp[i], (uint32_t)su[i], lt); },
        [&](uint32_t vi) { return KeyPair{load_stream4(bp + vi), load_stream4(bu + vi)}; },
        [&](const KeyPair(&kp)[kStarVecs], const bool(&valid)[kStarVecs]) {
          uint32_t w[4 * kStarVecs], p[4 * kStarVecs], u[4 * kStarVecs];
          bool pass[4 * kStarVecs];
#pragma unroll
          for (int v = 0; v < kStarVecs; ++v) {
            p[4 * v] = (uint32_t)kp[v].p.x, p[4 * v + 1] = (uint32_t)kp[v].p.y;
            p[4 * v + 2] = (uint32_t)kp[v].p.z, p[4 * v + 3] = (uint32_t)kp[v].p.w;
            u[4 * v] = (uint32_t)kp[v].u.x, u[4 * v + 1] = (uint32_t)kp[v].u.y;
            u[4 * v + 2] = (uint32_t)kp[v].u.z, u[4 * v + 3] = (uint32_t)kp[v].u.w;
          }
          uint32_t rare = 0;
#pragma unroll
          for (int i = 0; i < 4 * kStarVecs; ++i) {
            const bool in_c = u[i] < x.n_cust;
            pass[i] = valid[i / 4] && in_c && cust_pass<FULL>(x, u[i], lt);
            const uint32_t wp = prod_word(x, p[i], pass[i]);
            w[i] = pass[i] ? wp : kValid;
            rare |= (uint32_t)((pass[i] && wp == 0u) || (valid[i / 4] && (!in_c || p[i] >= x.n_prod)));
          }
#pragma unroll
          for (int i = 0; i < 4 * kStarVecs; ++i) star_add(a, w[i]);
          if (__builtin_expect(rare != 0u, 0)) {
#pragma unroll 1
            for (int i = 0; i < 4 * kStarVecs; ++i) {
              uint32_t pi = p[0], ui = u[0], wi = w[0];
              bool ps = pass[0], ok = valid[0];
#pragma unroll
              for (int j = 1; j < 4 * kStarVecs; ++j) {
                pi = i == j ? p[j] : pi;
                ui = i == j ? u[j] : ui;
                wi = i == j ? w[j] : wi;
                ps = i == j ? pass[j] : ps;
                ok = i == j ? valid[j / 4] : ok;
              }
              if ((ps && wi == 0u) || (ok && (ui >= x.n_cust || pi >= x.n_prod))) star_slow(a, x, pi, ui);
            }
          }
        });
    star_flush(a);
  }
  if (a.bad) *flag = 1;
}

template <typename K>
void allow_lds(K kernel, size_t bytes) {
  if (bytes > 48 * 1024)
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)bytes);
}

constexpr size_t kStaticReserve = 512;

}  // namespace

size_t star_lds_bytes(int32_t tp, int32_t tc, int32_t nq) {
  return (size_t)kStarBins * kWave * 8 + (size_t)((tp + 4) & ~3) * 4 + (size_t)((((tc + 31) / 32) + 4) & ~3) * 4 +
         (size_t)(nq + 1) * 4;
}

int32_t star_bits_stride(int32_t tc) { return (int32_t)(((((int64_t)tc + 31) / 32) + 3) & ~(int64_t)3); }

int32_t star_max_prod_hot(int32_t tc, int32_t nq, const DeviceInfo &dev) {
  const size_t fixed = star_lds_bytes(0, tc, nq) - 16 + kStaticReserve;
  if (dev.lds_per_block <= fixed + 16) return 0;
  return (int32_t)(((dev.lds_per_block - fixed) / 4) & ~(size_t)3) - 4;
}

int32_t star_max_cust_hot(int32_t nq, const DeviceInfo &dev) {
  // with an empty product prefix: bins, query table, reserve, and 16 bytes of padding per table
  const size_t fixed = star_lds_bytes(0, 0, nq) + 16 + kStaticReserve;
  if (dev.lds_per_block <= fixed) return 0;
  const size_t rows = ((dev.lds_per_block - fixed) / 16) * 128;  // whole 16-byte vectors of bits
  return (int32_t)(rows < (size_t)kStarMaxCustHot ? rows : (size_t)kStarMaxCustHot);
}

namespace {
size_t seg_padded(int32_t n_cust) { return ((size_t)n_cust + 31) / 32 * 32; }
}  // namespace

bool star_full_bits(int32_t n_cust, int32_t nq) {
  return (size_t)nq * (size_t)star_bits_stride(n_cust) * 4 <= kStarFullBitsBytes;
}

namespace {
// words per query bitmap: every customer row when all bitmaps fit the budget, else the largest LDS prefix
size_t star_bits_words(int32_t n_cust, int32_t nq) {
  if (star_full_bits(n_cust, nq)) return (size_t)star_bits_stride(n_cust);
  return (size_t)star_bits_stride(n_cust < kStarMaxCustHot ? n_cust : kStarMaxCustHot);
}
}  // namespace

size_t star_workspace_bytes(int32_t n_prod, int32_t n_cust, int32_t nq) {
  auto r = [](size_t x) { return (x + 255) & ~(size_t)255; };
  return r((size_t)n_prod * 4) + r(seg_padded(n_cust) + 16) + r((size_t)(nq + 1) * 4) + r(16) +
         r((size_t)nq * star_bits_words(n_cust, nq) * 4);
}

size_t star_workspace_bound(int32_t n_rows, int32_t nq) {
  // star_workspace_bytes(n_prod, n_cust, nq) for any n_prod, n_cust <= n_rows: the bitmaps of every customer
  // row take at most the budget when they are built, the LDS-prefix bitmaps otherwise
  auto r = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t full = (size_t)nq * (size_t)star_bits_stride(n_rows) * 4;
  const size_t prefix = (size_t)nq * (size_t)star_bits_stride(n_rows < kStarMaxCustHot ? n_rows : kStarMaxCustHot) * 4;
  const size_t bits = full < kStarFullBitsBytes ? full : kStarFullBitsBytes;
  return r((size_t)n_rows * 4) + r(seg_padded(n_rows) + 16) + r((size_t)(nq + 1) * 4) + r(16) +
         r(bits > prefix ? bits : prefix);
}

hipError_t launch_star(const int32_t *pkeys, const int32_t *ukeys, const int64_t *qstart, const int32_t *qlt,
                       int32_t nq, const int32_t *price, const int8_t *cat, int32_t n_prod, const int8_t *attr,
                       int32_t n_cust, int32_t tp, int32_t tc, int64_t tile_rows, int32_t blocks, int64_t *out_sum,
                       int64_t *out_cnt, int32_t *flag, void *ws, const DeviceInfo &dev, hipStream_t s) {
  auto r = [](size_t x) { return (x + 255) & ~(size_t)255; };
  char *w = (char *)ws;
  uint32_t *pwords = (uint32_t *)w;
  w += r((size_t)n_prod * 4);
  int8_t *cwords = (int8_t *)w;
  const int32_t attr_padded = (int32_t)seg_padded(n_cust);
  w += r((size_t)attr_padded + 16);
  uint32_t *tile_start = (uint32_t *)w;
  w += r((size_t)(nq + 1) * 4);
  uint32_t *counter = (uint32_t *)w;
  w += r(16);
  uint32_t *cbits = (uint32_t *)w;  // nq bitmaps of cstride words (16-byte aligned)
  const bool full = star_full_bits(n_cust, nq);
  const int32_t bit_rows = full ? n_cust : tc;  // rows every bitmap covers
  const int32_t cstride = star_bits_stride(bit_rows);
  if (tc < 0 || tc > n_cust || tc > kStarMaxCustHot) return hipErrorInvalidValue;

  StageTimer st = stage_begin("star_prep", s);
  const int64_t n_pack = n_prod > attr_padded ? n_prod : attr_padded;
  int64_t g = (n_pack + 255) / 256;
  if (g > (int64_t)dev.cu_count * 16) g = (int64_t)dev.cu_count * 16;
  hipLaunchKernelGGL(star_pack_kernel, dim3((int)(g > 0 ? g : 1)), dim3(256), 0, s, price, cat, n_prod, pwords, attr,
                     n_cust, cwords, attr_padded);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && bit_rows > 0) {
    const int32_t n_words = (int32_t)(((int64_t)bit_rows + 31) / 32);
    const dim3 grid((n_words + kBitsThreads - 1) / kBitsThreads, (nq + kBitsQueries - 1) / kBitsQueries);
    hipLaunchKernelGGL(star_bits_kernel, grid, dim3(kBitsThreads), 0, s, reinterpret_cast<const uint4 *>(cwords),
                       n_words, qlt, nq, cstride, cbits);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(star_plan_kernel, dim3(1), dim3(1024), 0, s, qstart, nq, tile_rows, tile_start, counter,
                       out_sum, out_cnt, flag);
    e = hipGetLastError();
  }
  stage_end(st, s);
  if (e != hipSuccess) return e;
  const size_t lds = star_lds_bytes(tp, tc, nq);
  auto kern = full ? star_batch_kernel<true> : star_batch_kernel<false>;
  allow_lds(kern, lds);
  st = stage_begin("star_batch", s);
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(kStarThreads), lds, s, pkeys, ukeys, qstart, qlt, nq,
                     tile_start, counter, tile_rows, pwords, n_prod, tp, (const uint32_t *)cwords, n_cust, tc, price,
                     cat, cbits, cstride, out_sum, out_cnt, flag);
  e = hipGetLastError();
  stage_end(st, s);
  return e;
}

}  // namespace skew

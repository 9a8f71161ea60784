// Pieces shared by the query kernels: the per-query dimension word, the
// bounds-checked record buffer, and the cold-item partition plan.
#pragma once

#include "device_common.h"

namespace skew {

// ---------------------------------------------------------------------------
// Per-query dimension word.  Section 3.2 builds, for each query, a copy of
// the dimension columns it needs in layout order; the two columns the query
// needs (price, category) and its predicate are packed into one 32-bit word
// per row, so a fact row costs one 4-byte read:
//   0x80000000 | (g + 1) << 25 | price   qualifies, group g, 0 <= price < 2^25
//   0x80000000                           does not qualify (or has no group)
//   0                                    qualifies, but the price does not fit:
//                                        a slow path reads the columns again
// A gather outside [0, n_rows) also reads 0 (buffer range check), so every
// zero word goes to the slow path, which tells the two cases apart.  Field
// (w >> 25) & 31 selects an accumulator bin; bin 0 is a sink never read back.
// ---------------------------------------------------------------------------
constexpr uint32_t kValid = 0x80000000u;
constexpr int kGroupShift = 25;
constexpr uint32_t kPriceMask = (1u << kGroupShift) - 1u;
constexpr int kJoinBins = 32;  // (w >> 25) & 31
constexpr int kJoinBinRows = 17;  // bins a word can select: 0 (sink) and 1..16 (groups)
constexpr int kCountShift = 44;  // a join bin packs count << 44 | sum
constexpr uint64_t kSumMask = (1ull << kCountShift) - 1ull;

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

// Structured buffer load: element `index` of a buffer of 4-byte records.  The
// hardware range check (index < num_records) returns 0 for any other index,
// negative keys included, without touching memory.
typedef int32_t rsrc_t __attribute__((ext_vector_type(4)));
__device__ uint32_t buffer_load_record(rsrc_t rsrc, int32_t vindex, int32_t voffset, int32_t soffset,
                                       int32_t aux) __asm("llvm.amdgcn.struct.buffer.load.i32");

// Structured buffer store of one 4-byte record; an index at or beyond the
// record count is dropped by the same range check.
__device__ void buffer_store_record(int32_t vdata, rsrc_t rsrc, int32_t vindex, int32_t voffset, int32_t soffset,
                                    int32_t aux) __asm("llvm.amdgcn.struct.buffer.store.i32");

__device__ __forceinline__ rsrc_t record_buffer(const void *base, uint32_t num_records) {
  const uint64_t a = (uint64_t)(uintptr_t)base;
  rsrc_t r;
  r.x = (int32_t)(uint32_t)a;
  r.y = (int32_t)(((uint32_t)(a >> 32) & 0xFFFFu) | (4u << 16));  // stride 4 bytes
  r.z = (int32_t)num_records;
  r.w = 0x00020000;  // gfx9 raw 32-bit data format
  return r;
}

// ---------------------------------------------------------------------------
// Cold-item partitioning (the second pass of the threshold split, Section
// 4.2.1).  Ids in [t, t + P * W) are cut into P slices of W = 2^w consecutive
// ids; slice p is small enough to live in LDS.  Pass 1 writes each block's
// cold items into its own segment and counts them per slice; a scan turns the
// (slice, block) counts into offsets; a scatter puts the items in slice
// order as 2-byte offsets inside their slice (W <= 2^16); pass 3 resolves
// the items of each slice from an LDS copy of it.
// ---------------------------------------------------------------------------
constexpr int kMaxSlices = 1024;

struct SliceTables {       // in global memory (workspace)
  uint32_t *hist;          // [P][B]: cold items of block b in slice p, then prefixes within the slice
  uint32_t *row_total;     // [P]: cold items of slice p
  uint32_t *total;         // [1]: number of cold items
  uint32_t *seg_count;     // [B]: cold items written by block b
  uint32_t *slice_off;     // [P + 1]: first item of slice p in slice order
};


// ---------------------------------------------------------------------------
// Cold-item compaction of pass 1.  Keys of the slots with cold[i] are
// appended to the workgroup's segment in slot order within the wave (one LDS
// reservation per 8 slots) and counted in their slice; the other lanes store
// out of range (dropped) and count into a sink word of their own, so the code
// has no per-slot branches.
// ---------------------------------------------------------------------------
struct ColdSink {
  uint32_t *count;  // LDS: items written so far
  uint32_t *hist;   // LDS [P + 64]: slice counts, then one sink word per lane
  uint32_t t;
  int32_t wshift;
  uint32_t sink;    // P + lane
  bool combine0 = false;  // count slice 0 with one add per slot (cold_append<..., true>)
};

// Number of lanes below this one in mask m.
__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// One LDS atomic per wave: the first active lane reserves n slots and the
// base is read back from that lane.
__device__ __forceinline__ uint32_t wave_reserve(uint32_t *count, uint32_t n) {
  const uint64_t act = __ballot(1);
  uint32_t base = 0;
  if ((uint32_t)lane_id() == (uint32_t)(__ffsll((unsigned long long)act) - 1)) base = atomicAdd(count, n);
  return __builtin_amdgcn_readfirstlane(base);
}

// store(i, idx) writes slot i at segment index idx (idx = -1: out of range).
// With COMBINE0 and o.combine0, the lanes of a slot whose keys fall into
// slice 0 (the densest one on a frequency-ordered layout) are counted by one
// LDS add instead of one each, so they do not queue on the same counter.
template <int N, class Store, bool COMBINE0 = false>
__device__ __forceinline__ void cold_append(const ColdSink &o, const uint32_t (&k)[N], const bool (&cold)[N],
                                            Store store) {
  constexpr int kPart = N < 8 ? N : 8;  // ballots live at once
#pragma unroll
  for (int p0 = 0; p0 < N; p0 += kPart) {
    uint64_t m[kPart];
    uint32_t total = 0;
#pragma unroll
    for (int i = 0; i < kPart; ++i) {
      m[i] = __ballot(cold[p0 + i]);
      total += (uint32_t)__popcll(m[i]);
    }
    if (total == 0) continue;
    uint32_t pos = wave_reserve(o.count, total);
#pragma unroll
    for (int i = 0; i < kPart; ++i) {
      const bool cd = cold[p0 + i];
      store(p0 + i, cd ? (int32_t)(pos + lanes_below(m[i])) : -1);
      const uint32_t sl = (k[p0 + i] - o.t) >> o.wshift;
      bool one = cd;
      if (COMBINE0 && o.combine0) {
        const bool z = cd && sl == 0;
        const uint64_t mz = __ballot(z);
        if (z && lanes_below(mz) == 0) lds_add_u32(&o.hist[0], (uint32_t)__popcll(mz));
        one = cd && !z;
      }
      lds_add_u32(&o.hist[one ? sl : o.sink], 1u);
      pos += (uint32_t)__popcll(m[i]);
    }
  }
}

// ---------------------------------------------------------------------------
// Dense form of the compaction, for a low cold share: the cold slots of a
// wave are moved by one lane permutation per slot into an open chunk of 64
// items held in registers (lane L holds item L of the chunk, NC columns); a
// full chunk takes one reservation and one dense store per column, so every
// store carries 64 items whatever the share of cold slots.  Items reach the
// segment in no particular order; the partition needs none.  Every lane of
// the wave must be active.
// ---------------------------------------------------------------------------
template <int NC>
struct WaveChunk {
  uint32_t col[NC];
  uint32_t n;  // items held, wave-uniform
};

// store(col, idx, ok): lanes with ok write their items at segment index idx.
template <int NC, class Store>
__device__ __forceinline__ void chunk_append(const ColdSink &o, WaveChunk<NC> &ch, bool cold,
                                             const uint32_t (&x)[NC], Store store) {
  const uint64_t m = __ballot(cold);
  const uint32_t n = (uint32_t)__popcll(m);
  if (n == 0) return;
  const uint32_t lane = lane_id();
  const uint32_t below = lanes_below(m);
  // cold lanes first, in lane order, then the others: a permutation of the
  // 64 lanes, rotated so that the cold items follow the open chunk
  const uint32_t rank = cold ? below : n + (lane - below);
  const int addr = (int)(((ch.n + rank) & (kWave - 1)) << 2);
  uint32_t y[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j) y[j] = (uint32_t)__builtin_amdgcn_ds_permute(addr, (int)x[j]);
  const uint32_t end = ch.n + n;
  const bool take = lane >= ch.n && lane < end;
#pragma unroll
  for (int j = 0; j < NC; ++j) ch.col[j] = take ? y[j] : ch.col[j];
  if (end >= (uint32_t)kWave) {
    const uint32_t pos = wave_reserve(o.count, kWave);
    store(ch.col, (int32_t)(pos + lane), true);
    const bool wrap = lane < end - kWave;
#pragma unroll
    for (int j = 0; j < NC; ++j) ch.col[j] = wrap ? y[j] : ch.col[j];
    ch.n = end - kWave;
  } else {
    ch.n = end;
  }
}

// The items left in the open chunk at the end of the workgroup's range.
template <int NC, class Store>
__device__ __forceinline__ void chunk_drain(const ColdSink &o, WaveChunk<NC> &ch, Store store) {
  if (ch.n == 0) return;
  const uint32_t pos = wave_reserve(o.count, ch.n);
  store(ch.col, (int32_t)(pos + lane_id()), (uint32_t)lane_id() < ch.n);
  ch.n = 0;
}

// ---------------------------------------------------------------------------
// Items [lo, hi) of item arrays that hold IPV items per 16-byte vector (and
// start 16-byte aligned at item 0), visited by a workgroup of THREADS
// threads: the items before the first vector boundary (threads 0..) and after
// the last one (threads 64..) one at a time, the rest in batches of V vectors
// per thread, the next batch loaded while the current one is processed, then
// one guarded partial batch.
//   one(i)                       item i
//   load(vi) -> T                vector vi (items IPV vi .. IPV vi + IPV - 1)
//   batch(const T (&)[V], const bool (&valid)[V])
// ---------------------------------------------------------------------------
template <int IPV, int V, int THREADS, class T, class One, class Load, class Batch>
__device__ __forceinline__ void walk_items(uint32_t lo, uint32_t hi, One one, Load load, Batch batch) {
  static_assert(IPV <= kWave, "head and tail items are taken by one wave each");
  const uint32_t al = (lo + IPV - 1) / IPV * IPV;
  if (al >= hi) {
    if (threadIdx.x < hi - lo) one(lo + threadIdx.x);
    return;
  }
  if (threadIdx.x < al - lo) one(lo + threadIdx.x);
  const uint32_t vb = al / IPV, ve = hi / IPV;
  if (threadIdx.x >= kWave && threadIdx.x - kWave < hi - IPV * ve) one(IPV * ve + threadIdx.x - kWave);

  constexpr uint32_t kBatch = (uint32_t)V * THREADS;
  const uint32_t full = vb + ((ve - vb) / kBatch) * kBatch;
  bool all_valid[V];
#pragma unroll
  for (int u = 0; u < V; ++u) all_valid[u] = true;
  auto fill = [&](T(&x)[V], uint32_t at) {
#pragma unroll
    for (int u = 0; u < V; ++u) x[u] = load(at + u * THREADS + threadIdx.x);
  };
  T xa[V], xb[V];
  uint32_t at = vb;
  if (at < full) fill(xa, at);
  while (at < full) {
    uint32_t nxt = at + kBatch;
    fill(xb, nxt < full ? nxt : at);  // unconditional: the last one re-reads the current batch
    batch(xa, all_valid);
    at = nxt;
    if (at >= full) break;
    nxt = at + kBatch;
    fill(xa, nxt < full ? nxt : at);
    batch(xb, all_valid);
    at = nxt;
  }
  if (full < ve) {
    T x[V];
    bool valid[V];
#pragma unroll
    for (int u = 0; u < V; ++u) {
      const uint32_t vi = full + u * THREADS + threadIdx.x;
      valid[u] = vi < ve;
      x[u] = load(valid[u] ? vi : vb);
    }
    batch(x, valid);
  }
}

// ---------------------------------------------------------------------------
// Share of workgroup b of B in pass 3.  Every slice costs its items plus S
// item-equivalents for copying or flushing its LDS image; the total cost is
// cut evenly and each cut is mapped back to an item (cuts inside a slice's
// fixed cost map to its first item).  soff[0..P] are the slice offsets.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t cost_to_item(const uint32_t *soff, int32_t P, uint32_t S, uint64_t c) {
  int32_t a = 0, z = P;  // largest p in [0, P] with soff[p] + p * S <= c
  while (a < z) {
    const int32_t m = (a + z + 1) >> 1;
    if ((uint64_t)soff[m] + (uint64_t)m * S <= c) a = m;
    else z = m - 1;
  }
  if (a == P) return soff[P];
  const uint64_t in = c - ((uint64_t)soff[a] + (uint64_t)a * S);
  return soff[a] + (in > S ? (uint32_t)(in - S) : 0u);
}

__device__ __forceinline__ void balanced_share(const uint32_t *soff, int32_t P, uint32_t S, uint32_t b, uint32_t B,
                                               uint32_t *lo, uint32_t *hi) {
  const uint64_t total = (uint64_t)soff[P] + (uint64_t)P * S;
  *lo = cost_to_item(soff, P, S, total * b / B);
  *hi = cost_to_item(soff, P, S, total * (b + 1) / B);
}

// Last slice that starts at or before item i (P >= 1).
__device__ __forceinline__ int32_t slice_of_item(const uint32_t *soff, int32_t P, uint32_t i) {
  int32_t a = 0, z = P - 1;
  while (a < z) {
    const int32_t m = (a + z + 1) >> 1;
    if (soff[m] <= i) a = m;
    else z = m - 1;
  }
  return a;
}

// Copy words [base, base + len) of a 4-byte column into LDS (16-byte loads
// when the source is 16-byte aligned at base).
__device__ __forceinline__ void stage_words(uint32_t *dst, const uint32_t *words, int64_t base, int32_t len) {
  const uint32_t *src = words + base;
  if (((uintptr_t)src & 15u) == 0) {
    const int nv = len >> 2;
    for (int i = threadIdx.x; i < nv; i += blockDim.x)
      reinterpret_cast<uint4 *>(dst)[i] = reinterpret_cast<const uint4 *>(src)[i];
    for (int i = 4 * nv + threadIdx.x; i < len; i += blockDim.x) dst[i] = src[i];
  } else {
    for (int i = threadIdx.x; i < len; i += blockDim.x) dst[i] = src[i];
  }
}

// Hot prefix + cold lookup state of the single-pass kernel.
struct HotCtx {
  const uint32_t *hot;  // LDS
  rsrc_t words;
  uint32_t t, tclamp;
};

__device__ __forceinline__ uint32_t fetch_hot_or_global(const HotCtx &h, uint32_t uk) {
  // Two reads without branching: a clamped LDS read and a buffer gather whose
  // index is pushed out of range for hot keys (it returns 0 and issues no
  // memory traffic); the select keeps the right one.
  const bool hot = uk < h.t;
  const uint32_t wl = h.hot[uk < h.tclamp ? uk : h.tclamp];
  const uint32_t wg = buffer_load_record(h.words, (int32_t)(hot ? 0xFFFFFFFFu : uk), 0, 0, 0);
  return hot ? wl : wg;
}

}  // namespace skew

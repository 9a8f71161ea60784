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
// order; pass 3 cuts every slice into units of at most kUnitItems items and
// resolves each unit from an LDS copy of its slice.
// ---------------------------------------------------------------------------
constexpr int kMaxSlices = 1024;
constexpr uint32_t kUnitItems = 1u << 16;

struct SliceTables {       // in global memory (workspace)
  uint32_t *hist;          // [P][B]: cold items of block b in slice p, then prefixes within the slice
  uint32_t *row_total;     // [P]: cold items of slice p
  uint32_t *total;         // [1]: number of cold items
  uint32_t *seg_count;     // [B]: cold items written by block b
  uint32_t *slice_off;     // [P + 1]: first item of slice p in slice order
  uint32_t *unit_start;    // [P + 1]: first unit of slice p
};

}  // namespace skew

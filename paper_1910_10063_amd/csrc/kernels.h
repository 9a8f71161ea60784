// Internal launch interface between the C ABI (skew_api.hip) and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace skew {

struct DeviceInfo {
  int device = -1;
  int cu_count = 0;
  size_t lds_per_block = 0;  // bytes of LDS one workgroup may use
};

// ---- layout build (Section 3.1 / 3.2) ----
constexpr int kSortTile = 4096;  // elements per radix-sort tile
inline int64_t sort_tiles(int64_t n) { return (n + kSortTile - 1) / kSortTile; }

hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s);
hipError_t launch_histogram(const int32_t *keys, int64_t n, int32_t n_keys, uint32_t *counts, int32_t *flag,
                            const DeviceInfo &dev, hipStream_t s);
// Stable sort of keys 0..n_keys-1 by (count desc, key asc).  Scratch: 4 arrays
// of n_keys u32 plus 256 * sort_tiles(n_keys) u32 of digit histograms.
hipError_t launch_rank_sort(const uint32_t *counts_by_key, int32_t n_keys, int64_t n_fact, int32_t *perm,
                            uint32_t *counts_by_rank, uint32_t *keys_a, uint32_t *keys_b, int32_t *vals_a,
                            int32_t *vals_b, uint32_t *digit_hist, uint32_t *scan_scratch, hipStream_t s);
hipError_t launch_inverse(const int32_t *perm, int32_t n, int32_t *rank, hipStream_t s);
hipError_t launch_permute_dims(const int32_t *perm, int32_t n, const int32_t *price, const int8_t *cat,
                               int32_t *price_out, int8_t *cat_out, hipStream_t s);
hipError_t launch_recode(const int32_t *keys, int64_t n, const int32_t *rank, const int32_t *perm, int32_t n_keys,
                         int32_t *out, const DeviceInfo &dev, hipStream_t s);
// Dimension rows [from, to) appended to a layout as its least frequent items.
hipError_t launch_append_rows(int32_t from, int32_t to, int32_t *perm, int32_t *rank, uint32_t *counts_by_rank,
                              const int32_t *price, const int8_t *cat, int32_t *price_out, int8_t *cat_out,
                              hipStream_t s);

// ---- prefix sums and cold-item partitioning ----
struct SliceTables;
// Exclusive prefix sum in place; `total` (nullable) receives the sum.  scratch
// (nullable, kScanBlocks words) lets large arrays use many workgroups.
constexpr int kScanBlocks = 512;
hipError_t launch_exclusive_scan(uint32_t *a, int64_t n, uint32_t *total, uint32_t *scratch, hipStream_t s);
// Scan of the (slice, block) counts and the slice table.
hipError_t launch_partition_plan(const SliceTables &tab, int32_t P, int32_t B, hipStream_t s);
// Move every block's cold items into slice order, as 2-byte offsets inside
// their slice (plus the values when seg_vals is given).
// combine0: blocks whose items are mostly in slice 0 (a frequency-ordered layout with a small or no hot
// prefix) rank those items with one LDS add per load.
constexpr int32_t kCombineBelow = 2048;  // hot prefixes below which the partitioned forms combine slice 0
hipError_t launch_partition_scatter(const SliceTables &tab, int32_t P, int32_t B, const int32_t *seg_keys,
                                    const int32_t *seg_vals, int64_t seg_cap, int32_t t, int32_t wshift,
                                    uint16_t *out_local, int32_t *out_vals, hipStream_t s, bool combine0 = false);
// The group-by's narrow records: group << kGroupNarrowShift | value in the
// segments, (group offset inside its slice) << kGroupNarrowShift | value in
// slice order (out_items), slices of 1 << wshift groups from group 0.
constexpr int kGroupNarrowShift = 12;
hipError_t launch_partition_scatter_narrow(const SliceTables &tab, int32_t P, int32_t B, const int32_t *seg_recs,
                                           int64_t seg_cap, int32_t wshift, int32_t *out_items, hipStream_t s,
                                           bool combine0 = false);

// Partitioned key histogram (large fact columns, at most kMaxSlices slices of
// 32768 keys).  counts must be zeroed; keys outside [0, n_keys) set *flag.
struct HistPlan {
  int32_t blocks, slices;
  int64_t round, seg_cap;
};
HistPlan hist_plan(int64_t n_fact, int32_t n_keys, const DeviceInfo &dev);
size_t hist_partition_bytes(const HistPlan &pl);
hipError_t launch_histogram_partitioned(const int32_t *keys, int64_t n_fact, int32_t n_keys, uint32_t *counts,
                                        int32_t *flag, void *part_ws, const HistPlan &pl, hipStream_t s);

// ---- queries (Section 4) ----
constexpr int kJoinThreads = 1024;
constexpr int kGroupThreads = 1024;
constexpr int kGroupCopies = 16;        // hottest ranks kept as per-lane copies (Section 4.2.2)
constexpr int kJoinSliceShift = 15;     // 32768 dimension words per LDS slice
constexpr int kGroupSliceShift = 13;    // 8192 groups per LDS slice
constexpr int64_t kMaxRound = 1LL << 28;         // keys per round of the partitioned key histogram
constexpr int64_t kJoinMaxRound = 1LL << 29;     // the join's rounds (fewer copies of each slice in pass 3)
constexpr int64_t kGroupMaxRound = 1LL << 29;    // the group-by's rounds
constexpr int64_t kPartitionMinFact = 1LL << 22;  // below this the single pass is used

// Partitioned form: cold items of each round go through per-block segments,
// a (slice, block) histogram, a scatter into slice order and a slice pass.
struct JoinPlan {
  int32_t blocks, wshift, slices;
  int64_t round, seg_cap;
};
using GroupPlan = JoinPlan;

size_t join_lds_bytes(int groups, int32_t hot_rows);
int32_t join_max_hot_rows(int groups, const DeviceInfo &dev);
JoinPlan join_plan(int64_t n_fact, int32_t n_rows, int32_t t, int groups, const DeviceInfo &dev);
size_t join_partition_bytes(const JoinPlan &pl);
// Prefix the join uses for these sizes and partition workspace; *partitioned
// tells which form runs.
int32_t join_hot_rows_used(int64_t n_fact, int32_t n_rows, int32_t by_cat, int32_t hot_rows, size_t part_bytes,
                           const DeviceInfo &dev, bool *partitioned);
size_t group_lds_bytes(int32_t hot_groups);
int32_t group_max_hot_groups(const DeviceInfo &dev);  // single pass
size_t group_split_lds_bytes(int32_t hot_groups, int32_t slices);
int32_t group_split_max_hot_groups(int32_t slices, const DeviceInfo &dev);  // partitioned form
GroupPlan group_plan(int64_t n_fact, int32_t n_groups, const DeviceInfo &dev);
int32_t group_narrow_slices(const GroupPlan &pl);  // record slices of the shared table (0: no records)
size_t group_partition_bytes(const GroupPlan &pl);

// part_ws/part_bytes: optional workspace for the partitioned form (NULL: single pass).
hipError_t launch_join(const int32_t *keys, int64_t n_fact, const int32_t *price, const int8_t *cat, int32_t n_rows,
                       int32_t cat_lt, int32_t by_cat, int32_t hot_rows, int64_t *out_sum, int64_t *out_cnt,
                       uint32_t *words, int32_t *flag, void *part_ws, size_t part_bytes, const DeviceInfo &dev,
                       hipStream_t s);

// ---- operator variants (Section 4.1) ----
int32_t materialize_max_hot_rows(const DeviceInfo &dev);
int64_t select_max_hot_rows(const DeviceInfo &dev);
int32_t heavy_max_lds_ranks(const DeviceInfo &dev);
size_t select_workspace_bytes(int64_t n_fact, int32_t n_rows, int32_t blocks);
hipError_t launch_materialize(const int32_t *keys, int64_t n, const int32_t *col, int32_t n_rows, int32_t t,
                              int32_t *out, int32_t *flag, const DeviceInfo &dev, hipStream_t s);
hipError_t launch_select(const int32_t *keys, int64_t n_fact, const int32_t *col, int32_t n_rows, int32_t lt,
                         int32_t t, int32_t *out, int64_t *count, int32_t *flag, void *ws, const DeviceInfo &dev,
                         hipStream_t s);
hipError_t launch_heavy(const int32_t *keys, int64_t n_fact, int32_t n_keys, int32_t k, const int32_t *perm,
                        int32_t *out_keys, int64_t *out_count, int32_t *flag, const DeviceInfo &dev, hipStream_t s);

// ---- stack-distance cache model (Section 3.3) ----
size_t model_workspace_bytes(int32_t n_keys, int32_t values_per_line);
hipError_t launch_cache_model(const uint32_t *counts_by_rank, int32_t n_keys, const int32_t *rank,
                              int32_t values_per_line, int64_t cache_lines, void *ws, double *out_hit,
                              const DeviceInfo &dev, hipStream_t s);

// ---- batched star join ----
constexpr int32_t kMaxStarQueries = 4096;
constexpr int32_t kStarMaxCustHot = 1 << 20;  // customer bitmap rows per query (128 KB)
constexpr size_t kStarFullBitsBytes = (size_t)1 << 30;  // all queries' bitmaps over every customer row
size_t star_lds_bytes(int32_t tp, int32_t tc, int32_t nq);
int32_t star_bits_stride(int32_t tc);
bool star_full_bits(int32_t n_cust, int32_t nq);
int32_t star_max_prod_hot(int32_t tc, int32_t nq, const DeviceInfo &dev);
int32_t star_max_cust_hot(int32_t nq, const DeviceInfo &dev);
size_t star_workspace_bytes(int32_t n_prod, int32_t n_cust, int32_t nq);
size_t star_workspace_bound(int32_t n_rows, int32_t nq);  // any n_prod, n_cust <= n_rows
hipError_t launch_star(const int32_t *pkeys, const int32_t *ukeys, const int64_t *qstart, const int32_t *qlt,
                       int32_t nq, const int32_t *price, const int8_t *cat, int32_t n_prod, const int8_t *attr,
                       int32_t n_cust, int32_t tp, int32_t tc, int64_t tile_rows, int32_t blocks, int64_t *out_sum,
                       int64_t *out_cnt, int32_t *flag, void *ws, const DeviceInfo &dev, hipStream_t s);

// ---- measurement ----
// One read pass over bytes (a multiple of 16) of a 16-byte aligned buffer;
// *out_sum (device) receives the 64-bit wrapping sum of its 32-bit words.
hipError_t launch_stream_probe(const void *buf, size_t bytes, uint64_t *out_sum, const DeviceInfo &dev,
                               hipStream_t s);

enum GroupMode { kGroupRange = 0, kGroupHash = 1, kGroupAtomic = 2 };
hipError_t launch_group(const int32_t *keys, const int32_t *vals, int64_t n_fact, int32_t n_groups, GroupMode mode,
                        int32_t hot_groups, const int32_t *perm, int64_t *out_sum, int64_t *out_cnt,
                        uint64_t *acc_sum, uint64_t *acc_cnt, int32_t *flag, void *part_ws, size_t part_bytes,
                        const DeviceInfo &dev, hipStream_t s);

}  // namespace skew

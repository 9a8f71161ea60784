/*
 * skew.h - C ABI of libskew.so: the frequency-ordered ("permutation index")
 * layout of Zhang and Ross, "Exploiting Data Skew for Improved Query
 * Performance", and the foreign-key join-aggregate and grouped aggregation
 * that run on it, as hand-written HIP kernels for gfx950 (MI355X).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every array argument is a DEVICE pointer on the current HIP device, owned
 *   by the caller, and must be 4-byte aligned (int8 columns: any alignment).
 *   The library allocates nothing: scratch space comes from the caller's
 *   `workspace` (device memory of at least skew_workspace_bytes(...) bytes,
 *   256-byte aligned).
 * - `stream` is a hipStream_t (NULL = the null stream).  Work is enqueued on it
 *   in order; unless stated otherwise a call returns without waiting.
 *   fk_join_aggregate, group_aggregate and star_join_batch enqueue kernels
 *   only (no memset or copy), so a caller may capture them in a HIP graph
 *   (with SKEW_CHECK unset, which adds a wait for the error flag).
 * - Keys and groups are 0-based offsets (Section 2.2: a foreign key is an
 *   array offset into the dimension table).
 * - All sums and counts are exact 64-bit integers (no floating point).
 *   Outputs are overwritten, never accumulated into.
 * - Arguments are checked on the host before any HIP call; a failed check
 *   returns SKEW_EINVAL or SKEW_ENOSPACE with no device work enqueued.
 * - Return value: SKEW_OK or a negative code below; skew_last_error() then
 *   holds a message.  Calls on distinct streams may run concurrently; calls
 *   that share a workspace must be ordered by the caller.
 */
#ifndef SKEW_H
#define SKEW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SKEW_OK 0
#define SKEW_EINVAL (-1)   /* null/misaligned pointer, negative size, bad parameter */
#define SKEW_ERANGE (-2)   /* a key or group id outside its domain was seen */
#define SKEW_ENOSPACE (-3) /* workspace smaller than skew_workspace_bytes(...) */
#define SKEW_EHIP (-4)     /* HIP runtime or launch failure */
#define SKEW_EDEVICE (-5)  /* no usable gfx950 device */

/* Operation ids for skew_workspace_bytes.  SKEW_OP_JOIN / SKEW_OP_GROUP give
 * the size that enables the partitioned form of the query (cold rows buffered,
 * partitioned by slice and resolved from LDS in a second pass) for inputs of
 * at least 2^22 rows; the *_SINGLE_PASS sizes are the minimum, with which the
 * single-pass kernels run.  A query uses the partitioned form whenever the
 * workspace it is given is large enough for it.  The join partitions at most
 * 1024 slices (2^25 dimension rows past the hot prefix) and gathers the keys of
 * any rows beyond them in its first pass; the group-by's partitioned form
 * needs n_groups <= 2^23 and larger domains run its single pass. */
#define SKEW_OP_BUILD 1
#define SKEW_OP_JOIN 2
#define SKEW_OP_GROUP 3
#define SKEW_OP_JOIN_SINGLE_PASS 4
#define SKEW_OP_GROUP_SINGLE_PASS 5
#define SKEW_OP_MATERIALIZE 6
#define SKEW_OP_SELECT 7
#define SKEW_OP_HEAVY 8
#define SKEW_OP_CACHE_MODEL 9 /* n_keys = keys; sized for lines of 1 value (the largest need) */
#define SKEW_OP_STAR 10       /* star_join_batch: n_fact = queries, n_keys = max(n_prod, n_cust) */

/* hot_rows / hot_groups special values. */
#define SKEW_HOT_AUTO (-1)  /* library picks the hot prefix: LDS capacity (the join
                               * takes less in its single pass on small inputs) */
#define SKEW_HOT_NONE (-2)  /* group_aggregate only: global atomics for every row */

/* Message of the last failed call on this thread ("" if none); valid until the
 * next call on the same thread. */
const char *skew_last_error(void);

/* Bytes of workspace the operation needs for n_fact fact rows and n_keys keys
 * (dimension rows for BUILD/JOIN, groups for GROUP).  Returns 0 for an unknown
 * op or negative sizes. */
size_t skew_workspace_bytes(int op, int64_t n_fact, int32_t n_keys);

/*
 * build_skew_layout - build the permutation index of one fact column and apply
 * it (Section 3.1, Section 3.2, Fig. 2).
 *
 *   fact_keys[n_fact]      int32 keys, each in [0, n_keys).
 *   n_keys                 dimension rows (>= 1); n_fact in [0, 2^32).
 *   dim_price[n_keys]      int32 dimension column to copy in the new order, or NULL.
 *   dim_category[n_keys]   int8 dimension column to copy in the new order, or NULL.
 *   perm[n_keys]           out: offset form, perm[r] = key with frequency rank r.
 *   rank[n_keys]           out: rank form (the "remap index"), rank[perm[r]] = r.
 *   counts_by_rank[n_keys] out (nullable): frequency of perm[r], non-increasing.
 *   fact_recoded[n_fact]   out (nullable): rank[fact_keys[j]]; may equal fact_keys
 *                          (recoded in place).
 *   price_out[n_keys]      out (NULL iff dim_price is NULL): dim_price[perm[r]].
 *   category_out[n_keys]   out (NULL iff dim_category is NULL): dim_category[perm[r]].
 *
 * Order: keys by decreasing frequency; equal frequencies by ascending key, so
 * the layout is unique (keys that never occur come last).  Steps: key
 * histogram, stable radix sort of keys by frequency, inversion, dimension
 * copy, fact recode.  The call waits once, after the histogram: if any key is
 * outside [0, n_keys) it returns SKEW_ERANGE and writes none of the outputs.
 * Otherwise the remaining steps are enqueued and the call returns at once.
 */
int build_skew_layout(const int32_t *fact_keys, int64_t n_fact, int32_t n_keys, const int32_t *dim_price,
                      const int8_t *dim_category, int32_t *perm, int32_t *rank, uint32_t *counts_by_rank,
                      int32_t *fact_recoded, int32_t *price_out, int8_t *category_out, void *workspace,
                      size_t workspace_bytes, void *stream);

/*
 * append_skew_layout - maintenance of a layout without a rebuild (Section
 * 3.1): dimension rows inserted after the build are appended to the
 * dimension and to the end of the permutation index as its least frequent
 * items, and fact rows inserted afterwards are recoded through the extended
 * index; their frequencies are not counted (the layout drifts from the true
 * order until it is rebuilt, and stays exact).
 *
 *   n_old, n_new           dimension rows before and after (1 <= n_old <= n_new).
 *   perm[n_new], rank[n_new]
 *                          in: the layout of the first n_old rows; out: rows
 *                          [n_old, n_new) get perm[i] = rank[i] = i.
 *   counts_by_rank[n_new]  nullable: 0 for the new ranks.
 *   dim_price[n_new], dim_category[n_new]
 *                          the dimension in its original order, new rows at the
 *                          end (each nullable, with its output).
 *   price_out[n_new], category_out[n_new]
 *                          the permuted copy; rows [n_old, n_new) are appended.
 *   fact_keys_new[n_fact_new]     new fact keys in [0, n_new) (original ids).
 *   fact_recoded_new[n_fact_new]  out: rank[fact_keys_new[j]] (may alias); a key
 *                          outside [0, n_new) is copied unchanged, and the
 *                          queries flag it.
 * Stream-ordered, no wait.  Needs no workspace.
 */
int append_skew_layout(int32_t n_old, int32_t n_new, int32_t *perm, int32_t *rank, uint32_t *counts_by_rank,
                       const int32_t *dim_price, const int8_t *dim_category, int32_t *price_out, int8_t *category_out,
                       const int32_t *fact_keys_new, int64_t n_fact_new, int32_t *fact_recoded_new, void *stream);

/*
 * fk_join_aggregate - foreign-key join of a fact column with a dimension table,
 * filtered and aggregated (Q1/Q2 of Section 1 feeding SUM and COUNT), with
 * threshold-based processing of the hot prefix (Section 4.2).
 *
 *   fact_keys[n_fact]     int32 keys into the dimension (identity layout: the
 *                         original keys; skew layout: fact_recoded).
 *   dim_price[n_rows]     int32 price column (same layout as the keys).
 *   dim_category[n_rows]  int8 category column.
 *   cat_lt                a fact qualifies when its row's category < cat_lt
 *                         (signed compare; cat_lt >= 128 means no filter).
 *   group_by_category     0: one output group; 1: 16 groups, group = category,
 *                         rows with category outside [0, 16) in no group.
 *   hot_rows              t: dimension rows [0, t) are hot (Section 4.2): the
 *                         first min(t, skew_max_hot_rows) of them are copied
 *                         into LDS once per workgroup and read from there; in
 *                         the partitioned form the hot rows past that capacity
 *                         are gathered from global memory (through the caches)
 *                         in pass 1, and the single pass clamps t to the
 *                         capacity.  0 = every row read from global memory
 *                         (the identity-layout method); SKEW_HOT_AUTO: the LDS
 *                         capacity.
 *   out_sum, out_count    out: int64[1] or int64[16].
 *   workspace             >= skew_workspace_bytes(SKEW_OP_JOIN_SINGLE_PASS, ...);
 *                         with skew_workspace_bytes(SKEW_OP_JOIN, n_fact, n_rows)
 *                         bytes the keys at or above t are buffered, partitioned
 *                         into slices of 32768 rows and resolved from LDS copies
 *                         of the slices (Section 4.2.1's second pass).
 *
 * Fact keys outside [0, n_rows) join nothing and set the workspace's error
 * flag (see skew_query_status).  The answer does not depend on t or on the
 * layout: the same query over (keys, dimension) and over (recoded keys,
 * permuted dimension) gives identical outputs.  With SKEW_CHECK=1 in the
 * environment the call waits and returns SKEW_ERANGE when the flag is set.
 */
int fk_join_aggregate(const int32_t *fact_keys, int64_t n_fact, const int32_t *dim_price,
                      const int8_t *dim_category, int32_t n_rows, int32_t cat_lt, int32_t group_by_category,
                      int32_t hot_rows, int64_t *out_sum, int64_t *out_count, void *workspace,
                      size_t workspace_bytes, void *stream);

/*
 * fk_join_aggregate_noalloc - fk_join_aggregate for callers that cannot
 * allocate device memory or pass a workspace: code under HIP graph capture,
 * serving loops and harnesses that forbid allocation.  Same arguments and
 * result as fk_join_aggregate without the workspace; it runs the single-pass
 * form.  Its scratch (the error flag and one packed 4-byte word per dimension
 * row) is a fixed array inside the library, one per device, held until the
 * process ends: n_rows above SKEW_NOALLOC_MAX_ROWS returns SKEW_EINVAL.  The
 * call allocates nothing.  Every call on a device shares that device's array,
 * which keeps the last call's contents (each call rewrites what it reads):
 * calls that overlap on one device, on different streams or threads, race,
 * and the caller must order them.  With SKEW_CHECK=1 the call waits and
 * returns SKEW_ERANGE when a key was outside [0, n_rows).
 */
#define SKEW_NOALLOC_MAX_ROWS (1 << 24) /* 64 MiB of words + 256 bytes per device */
int fk_join_aggregate_noalloc(const int32_t *fact_keys, int64_t n_fact, const int32_t *dim_price,
                              const int8_t *dim_category, int32_t n_rows, int32_t cat_lt, int32_t group_by_category,
                              int32_t hot_rows, int64_t *out_sum, int64_t *out_count, void *stream);

/*
 * group_aggregate - grouped SUM and COUNT (Q3 of Section 1) with hybrid
 * private/shared aggregation (Section 4.3) and per-lane copies of the hottest
 * groups (Section 4.2.2).
 *
 *   group_keys[n_fact]  int32 group ids in [0, n_groups) (skew layout: ranks).
 *   values[n_fact]      int32 values.
 *   n_groups            >= 1.
 *   hot_groups          t > 0: groups [0, t) are aggregated in per-workgroup LDS
 *                       bins (clamped to capacity); the rest are either
 *                       partitioned into slices of 8192 groups and summed in
 *                       LDS (workspace of SKEW_OP_GROUP size) or sent to global
 *                       atomics (single-pass workspace).  In the partitioned
 *                       form a bin takes rows with values in [0, 2^16); a hot
 *                       row with another value is partitioned like a cold one.
 *                       Partitioned rows with values in [0, 2^12) over at most
 *                       2^20 groups move as 4-byte records, the others as
 *                       (group, value) pairs; the results do not depend on
 *                       which.  0: no id-based
 *                       privatisation, the layout-oblivious method: every row
 *                       partitioned (large workspace) or an LDS hash table of
 *                       the first groups met (single pass).  SKEW_HOT_NONE:
 *                       global atomics only.  SKEW_HOT_AUTO: LDS capacity.
 *   perm[n_groups]      nullable.  If set, group_keys are ranks and the
 *                       outputs are returned in original-key order:
 *                       out[perm[r]] = aggregate of rank r.
 *   out_sum, out_count  out: int64[n_groups].
 *   workspace           >= skew_workspace_bytes(SKEW_OP_GROUP_SINGLE_PASS, ...);
 *                       SKEW_OP_GROUP size enables the partitioned form.
 *
 * Rows whose key is outside [0, n_groups) are skipped and set the error flag.
 */
int group_aggregate(const int32_t *group_keys, const int32_t *values, int64_t n_fact, int32_t n_groups,
                    int32_t hot_groups, const int32_t *perm, int64_t *out_sum, int64_t *out_count,
                    void *workspace, size_t workspace_bytes, void *stream);

/*
 * materialize_column - materialization (Q1 of Section 1, operator of Section
 * 4.1): out[j] = dim_col[fact_keys[j]] for j in [0, n_fact).
 *
 *   fact_keys[n_fact]  int32 keys (original keys with the original column, or
 *                      recoded keys with the permuted column).
 *   dim_col[n_rows]    int32 dimension column.
 *   hot_rows           rows [0, t) are copied into LDS once per workgroup and
 *                      read there (clamped to LDS capacity); 0 = every key
 *                      gathered from global memory; SKEW_HOT_AUTO.
 *   out[n_fact]        int32 output; may not overlap fact_keys.
 *   workspace          >= skew_workspace_bytes(SKEW_OP_MATERIALIZE, n_fact, n_rows).
 *
 * A key outside [0, n_rows) materializes 0 and sets the error flag.
 */
int materialize_column(const int32_t *fact_keys, int64_t n_fact, const int32_t *dim_col, int32_t n_rows,
                       int32_t hot_rows, int32_t *out, void *workspace, size_t workspace_bytes, void *stream);

/*
 * select_fact_rows - selection (Q2 of Section 1, operator of Section 4.1):
 * the offsets j of the fact rows with dim_col[fact_keys[j]] < lt, in
 * increasing order.  The predicate is evaluated once per dimension row into a
 * bitmap in the workspace; the bits of rows [0, hot_rows) are copied into
 * LDS (8 rows per LDS byte, clamped to capacity).
 *
 *   fact_keys[n_fact]   int32 keys, n_fact < 2^31.
 *   dim_col[n_rows]     int32 dimension column; lt: signed bound.
 *   hot_rows            as for materialize_column, counted in rows (bits).
 *   out_offsets[n_fact] int32 output (capacity for every row); the first
 *                       *out_count entries are written.
 *   out_count           int64[1] device output: number of offsets.
 *   workspace           >= skew_workspace_bytes(SKEW_OP_SELECT, n_fact, n_rows).
 *
 * Keys outside [0, n_rows) never qualify and set the error flag.
 */
int select_fact_rows(const int32_t *fact_keys, int64_t n_fact, const int32_t *dim_col, int32_t n_rows, int32_t lt,
                     int32_t hot_rows, int32_t *out_offsets, int64_t *out_count, void *workspace,
                     size_t workspace_bytes, void *stream);

/*
 * heavy_hitter_counts - Q3a of Section 1 on the frequency-ordered layout
 * (Section 4.2.2): the k most frequent keys are the ranks [0, k), so only
 * those are counted and every other row is dropped.
 *
 *   ranked_keys[n_fact] int32 recoded keys (ranks) in [0, n_keys).
 *   k                   number of heavy hitters, 0 <= k <= n_keys.
 *   perm[n_keys]        nullable: the permutation index; out_keys[r] = perm[r]
 *                       (original key of rank r), else out_keys[r] = r.
 *   out_keys[k]         int32 output.
 *   out_count[k]        int64 output: rows of rank r.
 *   workspace           >= skew_workspace_bytes(SKEW_OP_HEAVY, n_fact, n_keys).
 *
 * With a layout built on the same column, (out_keys, out_count) are the k most
 * frequent keys with their counts, most frequent first, equal counts by
 * ascending key.  Keys outside [0, n_keys) are dropped and set the error flag.
 */
int heavy_hitter_counts(const int32_t *ranked_keys, int64_t n_fact, int32_t n_keys, int32_t k, const int32_t *perm,
                        int32_t *out_keys, int64_t *out_count, void *workspace, size_t workspace_bytes,
                        void *stream);

/*
 * cache_model_hit_rate - the stack-distance cache model of Section 3.3: the
 * hit rate an LRU cache of cache_lines lines is expected to reach on the
 * dimension lookups of a fact column, for a given layout.  Line frequencies
 * come from the key frequencies (Section 3.3: with the frequency-ordered
 * layout the most frequent line holds the v most frequent values); for line
 * i the model finds the number of trials K_i after which S other distinct
 * lines are expected, and sums f_i (1 - (1 - f_i)^K_i).
 *
 *   counts_by_rank[n_keys]  uint32 frequencies in rank order (build_skew_layout).
 *   rank[n_keys]            nullable.  NULL: the frequency-ordered layout (line i
 *                           holds ranks [i v, (i + 1) v)).  Else the identity
 *                           layout: line i holds keys [i v, (i + 1) v), key k
 *                           occurring counts_by_rank[rank[k]] times.
 *   values_per_line         v >= 1 (32 for 128-byte lines of 4-byte values).
 *   cache_lines             S >= 1.
 *   out_hit                 HOST double: the modelled hit rate (0 with no lookups).
 *   workspace               >= skew_workspace_bytes(SKEW_OP_CACHE_MODEL, 0, n_keys).
 *
 * The sum of frequencies must be below 2^32.  The call waits for the stream.
 */
int cache_model_hit_rate(const uint32_t *counts_by_rank, int32_t n_keys, const int32_t *rank,
                         int32_t values_per_line, int64_t cache_lines, double *out_hit, void *workspace,
                         size_t workspace_bytes, void *stream);

/*
 * Batched star join: many fact
 * tables, each with a product key and a customer key per row, joined with a
 * product dimension (price, category) and a customer dimension (int8
 * segment).  Query q returns SUM(price) and COUNT(*) grouped by the product's
 * category (16 groups) over its rows whose customer has segment <
 * query_cust_lt[q].  It is the FK join-aggregate of Section 1 with a second,
 * filtering dimension; on frequency-ordered layouts of both dimensions
 * (Section 3, one layout per dimension built from all queries' keys) the hot
 * rows of each are the first ones and are read from LDS (Section 4.2).
 *
 * One persistent kernel takes tiles of tile_rows rows from a device work queue
 * (a tile never spans two queries), so queries of very different sizes share
 * the GPU.  Before it, a kernel evaluates every query's filter on the hot
 * customer rows into a per-query bitmap in the workspace; a workgroup stages
 * the bitmap of the query it works on into LDS.  Every launch of the call is
 * a kernel, so a caller may capture the call in a HIP graph and replay it.
 */
typedef struct {
  int32_t prod_hot_rows; /* product rows [0, t) read from LDS (clamped to capacity) */
  int32_t cust_hot_rows; /* customer rows [0, t) resolved from LDS, t <= 2^20: one bit
                            per row, the outcome of the query's filter */
  int32_t tile_rows;     /* rows per work-queue tile, in [1024, 2^24] */
  int32_t blocks;        /* persistent workgroups; 0 = one per compute unit */
} skew_star_tuning;

/*
 *   prod_keys[N], cust_keys[N]  int32 keys of all queries, one query after the
 *                               other (N = query_start[n_queries]); both
 *                               16-byte aligned.
 *   query_start[n_queries + 1]  int64 device array: query q owns rows
 *                               [query_start[q], query_start[q + 1]); non-decreasing.
 *   query_cust_lt[n_queries]    int32 device array: customer threshold of query q.
 *   n_queries                   1 .. 4096.
 *   prod_price[n_prod], prod_category[n_prod], cust_segment[n_cust].
 *   tuning                      host pointer; NULL = defaults (see star_join_autotune).
 *   out_sum, out_count          int64[n_queries * 16] (query-major).
 *   workspace                   >= skew_workspace_bytes(SKEW_OP_STAR, n_queries,
 *                               max(n_prod, n_cust)): packed product words
 *                               (4 bytes per row), a padded copy of the
 *                               segments, the work queue, and one bitmap per
 *                               query: over every customer row when the
 *                               n_queries bitmaps take at most 1 GiB, else over
 *                               min(n_cust, 2^20) rows.
 * Keys outside their dimension join nothing and set the error flag.
 */
int star_join_batch(const int32_t *prod_keys, const int32_t *cust_keys, const int64_t *query_start,
                    const int32_t *query_cust_lt, int32_t n_queries, const int32_t *prod_price,
                    const int8_t *prod_category, int32_t n_prod, const int8_t *cust_segment, int32_t n_cust,
                    const skew_star_tuning *tuning, int64_t *out_sum, int64_t *out_count, void *workspace,
                    size_t workspace_bytes, void *stream);

/*
 * star_join_autotune - the autotuner of star_join_batch: runs the batch with
 * each candidate split of LDS between the two hot prefixes, each tile size and
 * each persistent-workgroup count (one and two per compute unit), one warm-up
 * and three runs each timed with HIP events on `stream`, and writes the tuning
 * of the smallest median to *best and that median (ms) to *best_ms.  Same
 * arguments as star_join_batch (the outputs hold the last run's result).
 * Waits for the stream.
 */
int star_join_autotune(const int32_t *prod_keys, const int32_t *cust_keys, const int64_t *query_start,
                       const int32_t *query_cust_lt, int32_t n_queries, const int32_t *prod_price,
                       const int8_t *prod_category, int32_t n_prod, const int8_t *cust_segment, int32_t n_cust,
                       int64_t *out_sum, int64_t *out_count, skew_star_tuning *best, float *best_ms,
                       void *workspace, size_t workspace_bytes, void *stream);

/*
 * Threshold prior of the queries (Section 4.2: the hot rows are those the
 * cache holds; Section 3.3: the stack-distance model of the other lookups).
 * skew_join_choose and skew_group_choose read the frequencies of a layout
 * (counts_by_rank of build_skew_layout, device) and pick:
 *   hot_rows     the leading ranks, within the LDS capacity, whose keys would
 *                move more bytes through the cold path than copying the row
 *                into every workgroup costs;
 *   partitioned  1 when the partitioned form is modelled to move fewer HBM
 *                bytes than the single pass: pass a SKEW_OP_JOIN / SKEW_OP_GROUP
 *                workspace; 0: a *_SINGLE_PASS workspace.
 * and report the modelled quantities.  l2_hit is the model's LRU hit rate of
 * the lookups at or above hot_rows in one XCD's 4 MB L2 (32768 lines of 128
 * bytes; frequency-ordered lines of 32 dimension words, or of 16 groups'
 * 8-byte accumulators).  workspace >= skew_workspace_bytes(SKEW_OP_CACHE_MODEL,
 * 0, n_keys).  The calls wait for the stream.  The answer of the query never
 * depends on the choice.
 */
typedef struct {
  int32_t hot_rows;
  int32_t partitioned;
  double cold_share;        /* fact rows at or above hot_rows / n_fact */
  double l2_hit;            /* modelled L2 hit rate of those rows' lookups */
  double bytes_single;      /* modelled HBM bytes of the single pass */
  double bytes_partitioned; /* modelled HBM bytes of the partitioned form */
} skew_choice;
int skew_join_choose(const uint32_t *counts_by_rank, int32_t n_keys, int64_t n_fact, int32_t group_by_category,
                     skew_choice *out, void *workspace, size_t workspace_bytes, void *stream);
int skew_group_choose(const uint32_t *counts_by_rank, int32_t n_groups, int64_t n_fact, skew_choice *out,
                      void *workspace, size_t workspace_bytes, void *stream);

/*
 * skew_query_status - wait for `stream`, then report whether the last query
 * call that used this workspace saw an out-of-range key (SKEW_ERANGE) or not
 * (SKEW_OK).
 */
int skew_query_status(const void *workspace, size_t workspace_bytes, void *stream);

/*
 * stream_probe - measurement: one read pass over `bytes` of device memory
 * with 16-byte loads; *out_sum receives the 64-bit wrapping sum of its 32-bit
 * words (so no load can be skipped).  Timed by the caller, it gives the HBM
 * read rate a streaming kernel reaches on the device, the practical ceiling
 * beside the published peak for the query passes, which mostly read.
 *
 *   buf       device pointer, 16-byte aligned (NULL allowed when bytes = 0).
 *   bytes     multiple of 16.
 *   out_sum   device pointer to one uint64, overwritten.
 *
 * Stream-ordered.  SKEW_EINVAL for a NULL or misaligned pointer or a size
 * that is not a multiple of 16.
 */
int stream_probe(const void *buf, size_t bytes, uint64_t *out_sum, void *stream);

/* Stage timing, for benchmarks.  While enabled (on != 0), every launch stage
 * of the calls above (e.g. "join_pack", "join_split", "join_scatter", "join_slice",
 * "build_histogram") records a pair of HIP events on the stream it runs on.
 * skew_profile_report waits for them, writes up to max_stages entries (stage
 * names as consecutive NUL-terminated strings in names[names_bytes], total
 * milliseconds in ms[], number of launches in calls[]), forgets them, and
 * returns the number of entries.  Off by default; costs two events per stage. */
void skew_profile_enable(int on);
int skew_profile_report(char *names, int names_bytes, float *ms, int *calls, int max_stages);

/* Hot-prefix capacities (rows / groups) the kernels can hold in LDS on the
 * current device, or a negative code.  skew_max_hot_groups is the capacity
 * of the partitioned group-by (8 bytes per group; it may hold a few more when
 * there are fewer slices); the single pass holds fewer (12 bytes per group). */
int32_t skew_max_hot_rows(int32_t group_by_category);
/* The hot threshold fk_join_aggregate uses for these arguments (hot_rows as
 * the call takes it, workspace_bytes as passed to it): hot_rows clamped to
 * n_rows, and to skew_max_hot_rows in the single pass; with SKEW_HOT_AUTO,
 * the LDS capacity, and for the single pass over a small input a shorter
 * prefix (a workgroup would copy more rows than it looks up).  A negative
 * code on bad arguments. */
int32_t skew_join_hot_rows(int64_t n_fact, int32_t n_rows, int32_t group_by_category, int32_t hot_rows,
                           size_t workspace_bytes);
int32_t skew_max_hot_groups(void);
/* op: SKEW_OP_MATERIALIZE (rows), SKEW_OP_SELECT (rows, i.e. bits), SKEW_OP_HEAVY
 * (ranks counted in LDS; ranks in [capacity, k) use global atomics),
 * SKEW_OP_GROUP_SINGLE_PASS (hot groups of the single-pass group-by). */
int64_t skew_max_hot(int op);

#ifdef __cplusplus
}
#endif

#endif /* SKEW_H */

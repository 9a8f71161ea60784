/*
 * Plain CPU oracle for the skew-layout join-aggregate path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load or call this code; the product path
 * never does.  It shares no source with the GPU library.
 *
 * Everything here is the plain definition, written as one ordered loop per
 * step, in 64-bit integers (no floating point).  Where the paper leaves a
 * detail open, the reading taken is stated next to the code:
 *   - keys are 0-based offsets into the dimension table (the paper's figure
 *     counts from 1);
 *   - keys with equal frequency are ordered by ascending key, so the
 *     permutation index is unique;
 *   - keys that never occur in the fact column still get a position: they
 *     come last, in ascending key order, so the permuted dimension keeps
 *     every row.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

/*
 * Frequency of every dimension key in the fact column C: the aggregation
 * query that starts index building (Section 3.1; Q3 of Section 1).
 * Keys outside [0, n_keys) are not counted; their number is returned.
 */
int64_t oracle_key_counts(const int32_t *C, int64_t n_fact, int32_t n_keys, int64_t *cnt) {
  int64_t invalid = 0;
  for (int32_t k = 0; k < n_keys; ++k) cnt[k] = 0;
  for (int64_t j = 0; j < n_fact; ++j) {
    const int32_t k = C[j];
    if (k < 0 || k >= n_keys) {
      ++invalid;
      continue;
    }
    cnt[k] += 1;
  }
  return invalid;
}

typedef struct {
  int64_t cnt;
  int32_t key;
} freq_entry;

/* Decreasing frequency; equal frequencies by ascending key. */
static int by_decreasing_frequency(const void *pa, const void *pb) {
  const freq_entry *a = (const freq_entry *)pa, *b = (const freq_entry *)pb;
  if (a->cnt != b->cnt) return a->cnt > b->cnt ? -1 : 1;
  return (a->key > b->key) - (a->key < b->key);
}

/*
 * Permutation index (Section 3, Fig. 2a): the keys listed in decreasing
 * frequency order, perm[r] = key of rank r.  Its rank representation
 * (Fig. 2b) is the inverse, rank[perm[r]] = r; both are kept so lookups in
 * either direction are O(1) (Section 3).  Sorting the small key domain by
 * frequency is the second step of index building (Section 3.1).
 */
void oracle_permutation_index(const int64_t *cnt, int32_t n_keys, int32_t *perm, int32_t *rank) {
  freq_entry *e = (freq_entry *)malloc(sizeof(freq_entry) * (size_t)(n_keys > 0 ? n_keys : 1));
  for (int32_t k = 0; k < n_keys; ++k) {
    e[k].cnt = cnt[k];
    e[k].key = k;
  }
  qsort(e, (size_t)n_keys, sizeof(freq_entry), by_decreasing_frequency);
  for (int32_t r = 0; r < n_keys; ++r) perm[r] = e[r].key;
  for (int32_t r = 0; r < n_keys; ++r) rank[perm[r]] = r;
  free(e);
}

/*
 * Recoding of the fact column (Section 3.1, Fig. 2c -> 2d): every reference
 * to dimension row i is replaced by a reference to row Rank(i).  A key
 * outside [0, n_keys) is copied unchanged.
 */
void oracle_recode(const int32_t *C, int64_t n_fact, const int32_t *rank, int32_t n_keys, int32_t *C_new) {
  for (int64_t j = 0; j < n_fact; ++j) {
    const int32_t k = C[j];
    C_new[j] = (k >= 0 && k < n_keys) ? rank[k] : k;
  }
}

/*
 * Copy of a dimension column in permutation-index order (Section 3.2):
 * out[r] = col[perm[r]].
 */
void oracle_permute_i32(const int32_t *col, const int32_t *perm, int32_t n_keys, int32_t *out) {
  for (int32_t r = 0; r < n_keys; ++r) out[r] = col[perm[r]];
}

void oracle_permute_i8(const int8_t *col, const int32_t *perm, int32_t n_keys, int8_t *out) {
  for (int32_t r = 0; r < n_keys; ++r) out[r] = col[perm[r]];
}

/*
 * Foreign-key join followed by aggregation (Q1 and Q2 of Section 1 feeding a
 * SUM/COUNT): for each fact row j in order, the dimension row k = C[j] is
 * looked up by array offset (Section 2.2); it qualifies when its category is
 * below cat_lt (signed 8-bit compare).  With by_category = 0 every qualifying
 * row adds to group 0; otherwise it adds to group category, and rows whose
 * category lies outside [0, 16) belong to no group.  Fact keys outside
 * [0, n_rows) join nothing.  Sums and counts are exact 64-bit integers.
 * n_groups outputs are written: 1, or 16 when by_category is set.
 */
void oracle_fk_join_aggregate(const int32_t *C, int64_t n_fact, const int32_t *price, const int8_t *category,
                              int32_t n_rows, int32_t cat_lt, int32_t by_category, int64_t *sum,
                              int64_t *count) {
  const int n_groups = by_category ? 16 : 1;
  for (int g = 0; g < n_groups; ++g) {
    sum[g] = 0;
    count[g] = 0;
  }
  for (int64_t j = 0; j < n_fact; ++j) {
    const int32_t k = C[j];
    if (k < 0 || k >= n_rows) continue;
    const int32_t c = category[k];
    if (!(c < cat_lt)) continue;
    int g = 0;
    if (by_category) {
      if (c < 0 || c >= 16) continue;
      g = c;
    }
    sum[g] += (int64_t)price[k];
    count[g] += 1;
  }
}

/*
 * Grouped aggregation (Q3 of Section 1, with a SUM next to the COUNT):
 * sum[g] = sum of V[j] over rows with G[j] = g, count[g] = number of such
 * rows, for g in [0, n_groups).  Rows whose key is outside [0, n_groups)
 * are skipped; their number is returned.
 */
int64_t oracle_group_aggregate(const int32_t *G, const int32_t *V, int64_t n_fact, int32_t n_groups, int64_t *sum,
                               int64_t *count) {
  int64_t invalid = 0;
  for (int32_t g = 0; g < n_groups; ++g) {
    sum[g] = 0;
    count[g] = 0;
  }
  for (int64_t j = 0; j < n_fact; ++j) {
    const int32_t g = G[j];
    if (g < 0 || g >= n_groups) {
      ++invalid;
      continue;
    }
    sum[g] += (int64_t)V[j];
    count[g] += 1;
  }
  return invalid;
}

/*
 * The whole index build of Section 3.1 / 3.2 in the paper's order: count,
 * sort by frequency, invert, recode the fact column, and copy the dimension
 * columns in the new order.  counts_by_rank[r] = frequency of perm[r].
 * price/category (and their outputs) may be NULL when the dimension has no
 * columns to copy.  Returns the number of out-of-range keys.
 */
int64_t oracle_build_layout(const int32_t *C, int64_t n_fact, int32_t n_keys, const int32_t *price,
                            const int8_t *category, int32_t *perm, int32_t *rank, int64_t *counts_by_rank,
                            int32_t *C_new, int32_t *price_new, int8_t *category_new) {
  int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_keys > 0 ? n_keys : 1));
  const int64_t invalid = oracle_key_counts(C, n_fact, n_keys, cnt);
  oracle_permutation_index(cnt, n_keys, perm, rank);
  for (int32_t r = 0; r < n_keys; ++r) counts_by_rank[r] = cnt[perm[r]];
  oracle_recode(C, n_fact, rank, n_keys, C_new);
  if (price && price_new) oracle_permute_i32(price, perm, n_keys, price_new);
  if (category && category_new) oracle_permute_i8(category, perm, n_keys, category_new);
  free(cnt);
  return invalid;
}

/*
 * Maintenance of the permutation index without a rebuild (Section 3.1): a
 * dimension row inserted at the end of the dimension (ids n_old..n_new-1)
 * joins the end of the permutation index as the new least frequent item, so
 * Perm(i) = Rank(i) = i for it and its columns land at the end of the
 * permuted copy; fact rows inserted afterwards are recoded through the
 * extended rank form, their frequencies ignored.  perm/rank/price_new/
 * category_new hold the layout of the first n_old rows and have room for
 * n_new.  Returns the number of new fact keys outside [0, n_new) (copied
 * unchanged by the recode).
 */
int64_t oracle_append_layout(int32_t n_old, int32_t n_new, int32_t *perm, int32_t *rank, const int32_t *price,
                             const int8_t *category, int32_t *price_new, int8_t *category_new, const int32_t *C_add,
                             int64_t n_add, int32_t *C_add_new) {
  for (int32_t i = n_old; i < n_new; ++i) {
    perm[i] = i;
    rank[i] = i;
    if (price && price_new) price_new[i] = price[i];
    if (category && category_new) category_new[i] = category[i];
  }
  int64_t invalid = 0;
  for (int64_t j = 0; j < n_add; ++j) invalid += (C_add[j] < 0 || C_add[j] >= n_new);
  oracle_recode(C_add, n_add, rank, n_new, C_add_new);
  return invalid;
}

/*
 * Materialization (Q1 of Section 1, operator of Section 4.1): the dimension
 * column gathered through the foreign key, out[j] = col[C[j]].  A key outside
 * [0, n_rows) materializes 0; the number of such keys is returned.
 */
int64_t oracle_materialize(const int32_t *C, int64_t n_fact, const int32_t *col, int32_t n_rows, int32_t *out) {
  int64_t invalid = 0;
  for (int64_t j = 0; j < n_fact; ++j) {
    const int32_t k = C[j];
    if (k < 0 || k >= n_rows) {
      out[j] = 0;
      ++invalid;
      continue;
    }
    out[j] = col[k];
  }
  return invalid;
}

/*
 * Selection (Q2 of Section 1, operator of Section 4.1): the offsets j of the
 * fact rows whose dimension row satisfies col[C[j]] < lt, in increasing
 * order.  (The paper evaluates the dimension predicate once into a bitmap and
 * tests one bit per fact row; the plain definition tests the predicate.)
 * Keys outside [0, n_rows) never qualify.  Returns the number of offsets.
 */
int64_t oracle_select(const int32_t *C, int64_t n_fact, const int32_t *col, int32_t n_rows, int32_t lt,
                      int64_t *out) {
  int64_t n = 0;
  for (int64_t j = 0; j < n_fact; ++j) {
    const int32_t k = C[j];
    if (k < 0 || k >= n_rows) continue;
    if (col[k] < lt) out[n++] = j;
  }
  return n;
}

/*
 * Heavy hitters (Q3a of Section 1, Section 4.2.2): the k most frequent keys
 * of G with their counts, most frequent first, equal counts by ascending key
 * (k is clamped to n_keys).  Counting every key and sorting is the plain
 * definition; it is also what the paper's conventional method has to do.
 * Returns the clamped k.
 */
int32_t oracle_heavy_hitters(const int32_t *G, int64_t n_fact, int32_t n_keys, int32_t k, int32_t *keys,
                             int64_t *counts) {
  if (k > n_keys) k = n_keys;
  if (k < 0) k = 0;
  freq_entry *e = (freq_entry *)malloc(sizeof(freq_entry) * (size_t)(n_keys > 0 ? n_keys : 1));
  for (int32_t g = 0; g < n_keys; ++g) {
    e[g].cnt = 0;
    e[g].key = g;
  }
  for (int64_t j = 0; j < n_fact; ++j) {
    const int32_t g = G[j];
    if (g >= 0 && g < n_keys) e[g].cnt += 1;
  }
  qsort(e, (size_t)n_keys, sizeof(freq_entry), by_decreasing_frequency);
  for (int32_t r = 0; r < k; ++r) {
    keys[r] = e[r].key;
    counts[r] = e[r].cnt;
  }
  free(e);
  return k;
}

/*
 * Stack-distance cache model (Section 3.3), as the paper states it.  f[0..L)
 * are the access frequencies of the cache lines (summing to 1) and the LRU
 * cache holds S lines.  For line i the next reference is geometric with
 * success probability f_i; after k trials every other line j is expected
 * n_j = k f_j / (1 - f_i) times, so the expected number of distinct other
 * lines is d(k) = k - sum_{j != i} max(0, n_j - 1).  K_i is the smallest
 * integer k >= S with d(k) >= S (binary search), cdf_i = 1 - (1 - f_i)^K_i,
 * and the hit rate is sum_i f_i cdf_i.  A line for which d never reaches S
 * (fewer than S other lines can occur) always hits.
 *
 * Parity is not pinned to the paper, which prints no output of the model;
 * the tests pin it to closed forms and to an exact LRU simulation within the
 * 5 % error the paper reports.
 */
static double model_distinct(const double *f, int64_t L, int64_t i, double k) {
  const double scale = k / (1.0 - f[i]);
  double rep = 0.0;
  for (int64_t j = 0; j < L; ++j) {
    if (j == i) continue;
    const double n = scale * f[j];
    if (n > 1.0) rep += n - 1.0;
  }
  return k - rep;
}

double oracle_cache_model(const double *f, int64_t L, int64_t S) {
  double hit = 0.0;
  for (int64_t i = 0; i < L; ++i) {
    if (f[i] <= 0.0) continue;
    if (f[i] >= 1.0 || S >= L) {  /* no other line, or the cache holds every line */
      hit += f[i];
      continue;
    }
    /* d grows towards the number of other lines with nonzero frequency */
    int64_t others = 0;
    for (int64_t j = 0; j < L; ++j)
      if (j != i && f[j] > 0.0) ++others;
    if (others < S) {
      hit += f[i];
      continue;
    }
    int64_t lo = S, hi = S;
    while (model_distinct(f, L, i, (double)hi) < (double)S) {
      if (hi > ((int64_t)1 << 60)) break;
      hi *= 2;
    }
    if (model_distinct(f, L, i, (double)hi) < (double)S) {  /* not reached in range: a hit */
      hit += f[i];
      continue;
    }
    while (lo < hi) {  /* smallest k in [lo, hi] with d(k) >= S */
      const int64_t mid = lo + (hi - lo) / 2;
      if (model_distinct(f, L, i, (double)mid) >= (double)S) hi = mid;
      else lo = mid + 1;
    }
    hit += f[i] * (1.0 - pow(1.0 - f[i], (double)lo));
  }
  return hit;
}

/*
 * Star join of one fact table with two dimensions: the FK join-aggregate of
 * Section 1 with a second dimension that filters (the batched star-join
 * workload).  Fact row j has a product key P[j] and a customer key U[j]; it
 * qualifies when cust_attr[U[j]] < cust_lt (signed 8-bit compare) and then
 * adds price[P[j]] and 1 to group category[P[j]]; rows whose category lies
 * outside [0, 16) belong to no group, and keys outside their dimension join
 * nothing.  sum and count have 16 entries.
 */
void oracle_star_join(const int32_t *P, const int32_t *U, int64_t n, const int32_t *price, const int8_t *category,
                      int32_t n_prod, const int8_t *cust_attr, int32_t n_cust, int32_t cust_lt, int64_t *sum,
                      int64_t *count) {
  for (int g = 0; g < 16; ++g) {
    sum[g] = 0;
    count[g] = 0;
  }
  for (int64_t j = 0; j < n; ++j) {
    const int32_t p = P[j], u = U[j];
    if (p < 0 || p >= n_prod || u < 0 || u >= n_cust) continue;
    if (!(cust_attr[u] < cust_lt)) continue;
    const int32_t g = category[p];
    if (g < 0 || g >= 16) continue;
    sum[g] += (int64_t)price[p];
    count[g] += 1;
  }
}

// C ABI of libskew.so (declared in include/skew.h): argument checks on the
// host, workspace carving, device capabilities, and kernel launches on the
// caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>

#include "../../include/skew.h"
#include "device_common.h"
#include "kernels.h"
#include "profiler.h"
#include "query_common.h"

#include <vector>

namespace {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

int ok() {
  g_last_error.clear();
  return SKEW_OK;
}

int hip_fail(hipError_t e, const char *what) {
  return fail(SKEW_EHIP, "%s: %s", what, hipGetErrorString(e));
}

bool aligned4(const void *p) { return ((uintptr_t)p & 3u) == 0; }
bool aligned256(const void *p) { return ((uintptr_t)p & 255u) == 0; }

size_t round_up(size_t x) { return (x + 255) & ~(size_t)255; }

bool check_enabled() {
  static const bool on = [] {
    const char *v = std::getenv("SKEW_CHECK");
    return v && v[0] && std::strcmp(v, "0") != 0;
  }();
  return on;
}

// Device capabilities, queried once per device.
constexpr int kMaxDevices = 64;
std::once_flag g_dev_once[kMaxDevices];
skew::DeviceInfo g_dev[kMaxDevices];
int g_dev_status[kMaxDevices];

int device_info(skew::DeviceInfo *out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(SKEW_EDEVICE, "no HIP device: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(SKEW_EDEVICE, "device id %d out of range", dev);
  std::call_once(g_dev_once[dev], [dev] {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) {
      g_dev_status[dev] = SKEW_EDEVICE;
      return;
    }
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
      g_dev_status[dev] = SKEW_EDEVICE;
      return;
    }
    g_dev[dev].device = dev;
    g_dev[dev].cu_count = prop.multiProcessorCount;
    g_dev[dev].lds_per_block = prop.sharedMemPerBlock;
    g_dev_status[dev] = SKEW_OK;
  });
  if (g_dev_status[dev] != SKEW_OK)
    return fail(SKEW_EDEVICE, "device %d is not a usable gfx950 device", dev);
  *out = g_dev[dev];
  return SKEW_OK;
}

// Workspace layouts.  The first 256 bytes always hold the query error flag.
struct BuildWs {
  size_t counts, keys_a, keys_b, vals_a, vals_b, hist, scan, part, part_bytes, total;
};

skew::DeviceInfo sizing_device();

BuildWs build_ws(int64_t n_fact, int32_t n_keys) {
  BuildWs w;
  const size_t n4 = round_up((size_t)n_keys * 4);
  w.counts = skew::kFlagBytes;
  w.keys_a = w.counts + n4;
  w.keys_b = w.keys_a + n4;
  w.vals_a = w.keys_b + n4;
  w.vals_b = w.vals_a + n4;
  w.hist = w.vals_b + n4;
  w.scan = w.hist + round_up((size_t)256 * 4 * (size_t)skew::sort_tiles(n_keys));
  w.part = w.scan + round_up((size_t)(skew::kScanBlocks + 1) * 4);
  // the partitioned histogram, for large fact columns
  w.part_bytes = 0;
  const skew::HistPlan pl = skew::hist_plan(n_fact, n_keys, sizing_device());
  if (n_fact >= skew::kPartitionMinFact && pl.slices <= skew::kMaxSlices)
    w.part_bytes = round_up(skew::hist_partition_bytes(pl));
  w.total = w.part + w.part_bytes;
  return w;
}

// Workgroups of the partitioned form (segments are sized for this many).
constexpr int kPartBlocks = 256;

skew::DeviceInfo sizing_device() {
  skew::DeviceInfo d;
  d.cu_count = kPartBlocks;
  return d;
}

size_t join_ws(int32_t n_rows) { return skew::kFlagBytes + round_up((size_t)n_rows * 4); }

// Extra bytes for the partitioned join (0 when it would not be used).
size_t join_part_ws(int64_t n_fact, int32_t n_rows) {
  if (n_fact < skew::kPartitionMinFact) return 0;
  const skew::JoinPlan pl = skew::join_plan(n_fact, n_rows, 0, 16, sizing_device());
  if (pl.slices <= 0 || pl.slices > skew::kMaxSlices) return 0;
  return round_up(skew::join_partition_bytes(pl));
}

size_t group_ws(int32_t n_groups) { return skew::kFlagBytes + 2 * round_up((size_t)n_groups * 8); }

size_t group_part_ws(int64_t n_fact, int32_t n_groups) {
  if (n_fact < skew::kPartitionMinFact) return 0;
  const skew::GroupPlan pl = skew::group_plan(n_fact, n_groups, sizing_device());
  if (pl.slices <= 0 || pl.slices > skew::kMaxSlices) return 0;
  return round_up(skew::group_partition_bytes(pl));
}

skew::DeviceInfo part_device(const skew::DeviceInfo &dev) {
  skew::DeviceInfo d = dev;
  if (d.cu_count > kPartBlocks) d.cu_count = kPartBlocks;
  return d;
}

// Scratch of fk_join_aggregate_noalloc, for callers that cannot allocate: the
// error flag (first kFlagBytes) and the packed dimension words of up to
// SKEW_NOALLOC_MAX_ROWS rows.  Every device the library runs on holds its own
// copy until the process ends.  In host code `scratch` is a host-side stand-in:
// its device address comes from hipGetSymbolAddress, once per device.
constexpr size_t kScratchBytes = skew::kFlagBytes + (size_t)SKEW_NOALLOC_MAX_ROWS * 4;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::once_flag g_scratch_once[kMaxDevices];
void *g_scratch_ptr[kMaxDevices];
hipError_t g_scratch_err[kMaxDevices];

// Device address of this device's scratch; call with the device current.
int scratch_address(int dev, char **out) {
  std::call_once(g_scratch_once[dev], [dev] {
    void *p = nullptr;
    g_scratch_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_scratch_ptr[dev] = g_scratch_err[dev] == hipSuccess ? p : nullptr;
  });
  if (g_scratch_err[dev] != hipSuccess) return hip_fail(g_scratch_err[dev], "address of the library's scratch");
  if (!g_scratch_ptr[dev] || ((uintptr_t)g_scratch_ptr[dev] & 255u))
    return fail(SKEW_EHIP, "the library's scratch has no 256-byte aligned device address");
  *out = (char *)g_scratch_ptr[dev];
  return SKEW_OK;
}

int read_flag(const void *workspace, hipStream_t s) {
  int32_t flag = 0;
  hipError_t e = hipMemcpyAsync(&flag, workspace, sizeof flag, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "reading the error flag");
  return flag ? fail(SKEW_ERANGE, "a key outside its domain was seen") : ok();
}

}  // namespace


// ---------------------------------------------------------------------------
// Stage timing: while enabled, every launch stage records a pair of HIP events
// on the stream it runs on; skew_profile_report resolves them.
// ---------------------------------------------------------------------------
namespace {
struct StageRecord {
  const char *name;
  hipEvent_t start, stop;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<StageRecord> g_prof;
}  // namespace

namespace skew {

StageTimer stage_begin(const char *name, hipStream_t s) {
  StageTimer t;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (!g_prof_on) return t;
  StageRecord r{name, nullptr, nullptr};
  if (hipEventCreate(&r.start) != hipSuccess || hipEventCreate(&r.stop) != hipSuccess) return t;
  if (hipEventRecord(r.start, s) != hipSuccess) return t;
  g_prof.push_back(r);
  t.slot = (int)g_prof.size() - 1;
  return t;
}

void stage_end(const StageTimer &t, hipStream_t s) {
  if (t.slot < 0) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (t.slot < (int)g_prof.size()) (void)hipEventRecord(g_prof[t.slot].stop, s);
}

}  // namespace skew

extern "C" {

const char *skew_last_error(void) { return g_last_error.c_str(); }

size_t skew_workspace_bytes(int op, int64_t n_fact, int32_t n_keys) {
  if (n_fact < 0 || n_keys < 0) return 0;
  switch (op) {
    case SKEW_OP_BUILD:
      return build_ws(n_fact, n_keys).total;
    case SKEW_OP_JOIN:
      return join_ws(n_keys) + join_part_ws(n_fact, n_keys);
    case SKEW_OP_GROUP:
      return group_ws(n_keys) + group_part_ws(n_fact, n_keys);
    case SKEW_OP_JOIN_SINGLE_PASS:
      return join_ws(n_keys);
    case SKEW_OP_GROUP_SINGLE_PASS:
      return group_ws(n_keys);
    case SKEW_OP_MATERIALIZE:
    case SKEW_OP_HEAVY:
      return skew::kFlagBytes;
    case SKEW_OP_CACHE_MODEL:
      return skew::kFlagBytes + round_up(skew::model_workspace_bytes(n_keys, 1));
    case SKEW_OP_STAR:
      return skew::kFlagBytes + round_up(skew::star_workspace_bound(n_keys, (int32_t)n_fact));
    case SKEW_OP_SELECT:
      return skew::kFlagBytes + round_up(skew::select_workspace_bytes(n_fact, n_keys, kPartBlocks));
    default:
      return 0;
  }
}

int build_skew_layout(const int32_t *fact_keys, int64_t n_fact, int32_t n_keys, const int32_t *dim_price,
                      const int8_t *dim_category, int32_t *perm, int32_t *rank, uint32_t *counts_by_rank,
                      int32_t *fact_recoded, int32_t *price_out, int8_t *category_out, void *workspace,
                      size_t workspace_bytes, void *stream) {
  if (n_fact < 0 || n_fact >= (int64_t)1 << 32) return fail(SKEW_EINVAL, "n_fact must be in [0, 2^32)");
  if (n_keys < 1) return fail(SKEW_EINVAL, "n_keys must be >= 1");
  if (n_fact > 0 && !fact_keys) return fail(SKEW_EINVAL, "fact_keys is NULL");
  if (!perm || !rank) return fail(SKEW_EINVAL, "perm and rank are required");
  if (!workspace) return fail(SKEW_EINVAL, "workspace is NULL");
  if ((dim_price == nullptr) != (price_out == nullptr))
    return fail(SKEW_EINVAL, "dim_price and price_out must both be set or both be NULL");
  if ((dim_category == nullptr) != (category_out == nullptr))
    return fail(SKEW_EINVAL, "dim_category and category_out must both be set or both be NULL");
  if (!aligned4(fact_keys) || !aligned4(perm) || !aligned4(rank) || !aligned4(counts_by_rank) ||
      !aligned4(fact_recoded) || !aligned4(dim_price) || !aligned4(price_out))
    return fail(SKEW_EINVAL, "32-bit arrays must be 4-byte aligned");
  if (!aligned256(workspace)) return fail(SKEW_EINVAL, "workspace must be 256-byte aligned");
  const BuildWs w = build_ws(n_fact, n_keys);
  if (workspace_bytes < w.total)
    return fail(SKEW_ENOSPACE, "workspace has %zu bytes, needs %zu", workspace_bytes, w.total);

  skew::DeviceInfo dev;
  if (int rc = device_info(&dev)) return rc;
  const hipStream_t s = (hipStream_t)stream;
  char *ws = (char *)workspace;
  int32_t *flag = (int32_t *)ws;
  uint32_t *counts = (uint32_t *)(ws + w.counts);

  // 1. key histogram (aggregation Q3), then wait once to validate the keys.
  skew::StageTimer st = skew::stage_begin("build_histogram", s);
  hipError_t e = skew::launch_fill_u32((uint32_t *)flag, 1, 0u, s);
  if (e == hipSuccess) e = skew::launch_fill_u32(counts, n_keys, 0u, s);
  if (e == hipSuccess) {
    const skew::DeviceInfo pdev = part_device(dev);
    const skew::HistPlan pl = skew::hist_plan(n_fact, n_keys, pdev);
    if (w.part_bytes > 0 && skew::hist_partition_bytes(pl) <= w.part_bytes)
      e = skew::launch_histogram_partitioned(fact_keys, n_fact, n_keys, counts, flag, ws + w.part, pl, s);
    else
      e = skew::launch_histogram(fact_keys, n_fact, n_keys, counts, flag, dev, s);
  }
  skew::stage_end(st, s);
  if (e != hipSuccess) return hip_fail(e, "histogram launch");
  int32_t bad = 0;
  e = hipMemcpyAsync(&bad, flag, sizeof bad, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "histogram");
  if (bad) return fail(SKEW_ERANGE, "a fact key lies outside [0, %d)", n_keys);

  // 2. sort keys by frequency, 3. invert, 4. copy the dimension, 5. recode the facts.
  st = skew::stage_begin("build_rank_sort", s);
  e = skew::launch_rank_sort(counts, n_keys, n_fact, perm, counts_by_rank, (uint32_t *)(ws + w.keys_a),
                             (uint32_t *)(ws + w.keys_b), (int32_t *)(ws + w.vals_a), (int32_t *)(ws + w.vals_b),
                             (uint32_t *)(ws + w.hist), (uint32_t *)(ws + w.scan), s);
  skew::stage_end(st, s);
  st = skew::stage_begin("build_inverse", s);
  if (e == hipSuccess) e = skew::launch_inverse(perm, n_keys, rank, s);
  skew::stage_end(st, s);
  st = skew::stage_begin("build_permute_dims", s);
  if (e == hipSuccess) e = skew::launch_permute_dims(perm, n_keys, dim_price, dim_category, price_out, category_out, s);
  skew::stage_end(st, s);
  st = skew::stage_begin("build_recode", s);
  if (e == hipSuccess && fact_recoded) e = skew::launch_recode(fact_keys, n_fact, rank, perm, n_keys, fact_recoded, dev, s);
  skew::stage_end(st, s);
  if (e != hipSuccess) return hip_fail(e, "layout launch");
  return ok();
}

namespace {

// Argument checks shared by the two join entry points (everything but the workspace).
int join_check(const int32_t *fact_keys, int64_t n_fact, const int32_t *dim_price, const int8_t *dim_category,
               int32_t n_rows, int32_t group_by_category, int32_t hot_rows, const int64_t *out_sum,
               const int64_t *out_count) {
  if (n_fact < 0) return fail(SKEW_EINVAL, "n_fact must be >= 0");
  if (n_rows < 1) return fail(SKEW_EINVAL, "n_rows must be >= 1");
  if (n_fact > 0 && !fact_keys) return fail(SKEW_EINVAL, "fact_keys is NULL");
  if (!dim_price || !dim_category) return fail(SKEW_EINVAL, "dimension columns are required");
  if (!out_sum || !out_count) return fail(SKEW_EINVAL, "outputs are required");
  if (group_by_category != 0 && group_by_category != 1) return fail(SKEW_EINVAL, "group_by_category must be 0 or 1");
  if (hot_rows < SKEW_HOT_AUTO) return fail(SKEW_EINVAL, "hot_rows must be >= 0 or SKEW_HOT_AUTO");
  if (!aligned4(fact_keys) || !aligned4(dim_price) || !aligned4(out_sum) || !aligned4(out_count))
    return fail(SKEW_EINVAL, "32/64-bit arrays must be 4-byte aligned");
  if (((uintptr_t)out_sum & 7u) || ((uintptr_t)out_count & 7u))
    return fail(SKEW_EINVAL, "outputs must be 8-byte aligned");
  return SKEW_OK;
}

}  // namespace

int append_skew_layout(int32_t n_old, int32_t n_new, int32_t *perm, int32_t *rank, uint32_t *counts_by_rank,
                       const int32_t *dim_price, const int8_t *dim_category, int32_t *price_out, int8_t *category_out,
                       const int32_t *fact_keys_new, int64_t n_fact_new, int32_t *fact_recoded_new, void *stream) {
  if (n_old < 1 || n_new < n_old) return fail(SKEW_EINVAL, "need 1 <= n_old <= n_new");
  if (n_fact_new < 0) return fail(SKEW_EINVAL, "n_fact_new must be >= 0");
  if (!perm || !rank) return fail(SKEW_EINVAL, "perm and rank are required");
  if ((dim_price == nullptr) != (price_out == nullptr))
    return fail(SKEW_EINVAL, "dim_price and price_out must both be set or both be NULL");
  if ((dim_category == nullptr) != (category_out == nullptr))
    return fail(SKEW_EINVAL, "dim_category and category_out must both be set or both be NULL");
  if (n_fact_new > 0 && (!fact_keys_new || !fact_recoded_new))
    return fail(SKEW_EINVAL, "fact_keys_new and fact_recoded_new are required");
  if (!aligned4(perm) || !aligned4(rank) || !aligned4(counts_by_rank) || !aligned4(dim_price) || !aligned4(price_out) ||
      !aligned4(fact_keys_new) || !aligned4(fact_recoded_new))
    return fail(SKEW_EINVAL, "32-bit arrays must be 4-byte aligned");
  skew::DeviceInfo dev;
  if (int rc = device_info(&dev)) return rc;
  const hipStream_t s = (hipStream_t)stream;
  hipError_t e = skew::launch_append_rows(n_old, n_new, perm, rank, counts_by_rank, dim_price, dim_category,
                                          price_out, category_out, s);
  if (e == hipSuccess)
    e = skew::launch_recode(fact_keys_new, n_fact_new, rank, perm, n_new, fact_recoded_new, dev, s);
  if (e != hipSuccess) return hip_fail(e, "append launch");
  return ok();
}

int fk_join_aggregate(const int32_t *fact_keys, int64_t n_fact, const int32_t *dim_price,
                      const int8_t *dim_category, int32_t n_rows, int32_t cat_lt, int32_t group_by_category,
                      int32_t hot_rows, int64_t *out_sum, int64_t *out_count, void *workspace,
                      size_t workspace_bytes, void *stream) {
  if (int rc = join_check(fact_keys, n_fact, dim_price, dim_category, n_rows, group_by_category, hot_rows, out_sum,
                          out_count))
    return rc;
  if (!workspace) return fail(SKEW_EINVAL, "workspace is NULL");
  if (!aligned256(workspace)) return fail(SKEW_EINVAL, "workspace must be 256-byte aligned");
  const size_t need = join_ws(n_rows);
  if (workspace_bytes < need) return fail(SKEW_ENOSPACE, "workspace has %zu bytes, needs %zu", workspace_bytes, need);

  skew::DeviceInfo dev;
  if (int rc = device_info(&dev)) return rc;
  const hipStream_t s = (hipStream_t)stream;
  char *ws = (char *)workspace;
  void *part = workspace_bytes > need ? (void *)(ws + need) : nullptr;
  const hipError_t e = skew::launch_join(fact_keys, n_fact, dim_price, dim_category, n_rows, cat_lt,
                                         group_by_category, hot_rows, out_sum, out_count,
                                         (uint32_t *)(ws + skew::kFlagBytes), (int32_t *)ws, part,
                                         part ? workspace_bytes - need : 0, part_device(dev), s);
  if (e != hipSuccess) return hip_fail(e, "join launch");
  if (check_enabled()) return read_flag(workspace, s);
  return ok();
}

int fk_join_aggregate_noalloc(const int32_t *fact_keys, int64_t n_fact, const int32_t *dim_price,
                              const int8_t *dim_category, int32_t n_rows, int32_t cat_lt, int32_t group_by_category,
                              int32_t hot_rows, int64_t *out_sum, int64_t *out_count, void *stream) {
  if (int rc = join_check(fact_keys, n_fact, dim_price, dim_category, n_rows, group_by_category, hot_rows, out_sum,
                          out_count))
    return rc;
  if (n_rows > SKEW_NOALLOC_MAX_ROWS)
    return fail(SKEW_EINVAL, "n_rows %d exceeds the %d rows the library's fixed scratch holds", n_rows,
                SKEW_NOALLOC_MAX_ROWS);
  skew::DeviceInfo dev;
  if (int rc = device_info(&dev)) return rc;
  char *ws = nullptr;
  if (int rc = scratch_address(dev.device, &ws)) return rc;
  const hipStream_t s = (hipStream_t)stream;
  // The pack kernel clears the flag and the outputs and rewrites every word the query reads.
  const hipError_t e = skew::launch_join(fact_keys, n_fact, dim_price, dim_category, n_rows, cat_lt,
                                         group_by_category, hot_rows, out_sum, out_count,
                                         (uint32_t *)(ws + skew::kFlagBytes), (int32_t *)ws, nullptr, 0,
                                         part_device(dev), s);
  if (e != hipSuccess) return hip_fail(e, "join launch");
  if (check_enabled()) return read_flag(ws, s);
  return ok();
}

int group_aggregate(const int32_t *group_keys, const int32_t *values, int64_t n_fact, int32_t n_groups,
                    int32_t hot_groups, const int32_t *perm, int64_t *out_sum, int64_t *out_count, void *workspace,
                    size_t workspace_bytes, void *stream) {
  if (n_fact < 0) return fail(SKEW_EINVAL, "n_fact must be >= 0");
  if (n_groups < 1) return fail(SKEW_EINVAL, "n_groups must be >= 1");
  if (n_fact > 0 && (!group_keys || !values)) return fail(SKEW_EINVAL, "group_keys and values are required");
  if (!out_sum || !out_count) return fail(SKEW_EINVAL, "outputs are required");
  if (!workspace) return fail(SKEW_EINVAL, "workspace is NULL");
  if (hot_groups < SKEW_HOT_NONE) return fail(SKEW_EINVAL, "hot_groups must be >= 0, SKEW_HOT_AUTO or SKEW_HOT_NONE");
  if (!aligned4(group_keys) || !aligned4(values) || !aligned4(perm))
    return fail(SKEW_EINVAL, "32-bit arrays must be 4-byte aligned");
  if (((uintptr_t)out_sum & 7u) || ((uintptr_t)out_count & 7u))
    return fail(SKEW_EINVAL, "outputs must be 8-byte aligned");
  if (!aligned256(workspace)) return fail(SKEW_EINVAL, "workspace must be 256-byte aligned");
  const size_t need = group_ws(n_groups);
  if (workspace_bytes < need) return fail(SKEW_ENOSPACE, "workspace has %zu bytes, needs %zu", workspace_bytes, need);

  skew::DeviceInfo dev;
  if (int rc = device_info(&dev)) return rc;
  skew::GroupMode mode = skew::kGroupRange;
  int32_t t = hot_groups;
  if (hot_groups == SKEW_HOT_NONE) {
    mode = skew::kGroupAtomic;
    t = 0;
  } else if (hot_groups == 0) {
    mode = skew::kGroupHash;
    if (dev.lds_per_block < 128 * 1024) return fail(SKEW_EDEVICE, "hash privatisation needs 128 KB of LDS");
  } else if (hot_groups == SKEW_HOT_AUTO) {
    t = INT32_MAX;  // clamped to the LDS capacity of the form that runs
  }
  const hipStream_t s = (hipStream_t)stream;
  char *ws = (char *)workspace;
  const size_t acc = round_up((size_t)n_groups * 8);
  void *part = workspace_bytes > need ? (void *)(ws + need) : nullptr;
  const hipError_t e = skew::launch_group(group_keys, values, n_fact, n_groups, mode, t, perm, out_sum, out_count,
                                          (uint64_t *)(ws + skew::kFlagBytes),
                                          (uint64_t *)(ws + skew::kFlagBytes + acc), (int32_t *)ws, part,
                                          part ? workspace_bytes - need : 0, part_device(dev), s);
  if (e != hipSuccess) return hip_fail(e, "group launch");
  if (check_enabled()) return read_flag(workspace, s);
  return ok();
}

int materialize_column(const int32_t *fact_keys, int64_t n_fact, const int32_t *dim_col, int32_t n_rows,
                       int32_t hot_rows, int32_t *out, void *workspace, size_t workspace_bytes, void *stream) {
  if (n_fact < 0) return fail(SKEW_EINVAL, "n_fact must be >= 0");
  if (n_rows < 1) return fail(SKEW_EINVAL, "n_rows must be >= 1");
  if (n_fact > 0 && (!fact_keys || !out)) return fail(SKEW_EINVAL, "fact_keys and out are required");
  if (!dim_col) return fail(SKEW_EINVAL, "dim_col is NULL");
  if (!workspace) return fail(SKEW_EINVAL, "workspace is NULL");
  if (hot_rows < SKEW_HOT_AUTO) return fail(SKEW_EINVAL, "hot_rows must be >= 0 or SKEW_HOT_AUTO");
  if (!aligned4(fact_keys) || !aligned4(dim_col) || !aligned4(out))
    return fail(SKEW_EINVAL, "32-bit arrays must be 4-byte aligned");
  if (n_fact > 0 && out + n_fact > fact_keys && fact_keys + n_fact > out)
    return fail(SKEW_EINVAL, "out overlaps fact_keys");
  if (!aligned256(workspace)) return fail(SKEW_EINVAL, "workspace must be 256-byte aligned");
  if (workspace_bytes < skew::kFlagBytes)
    return fail(SKEW_ENOSPACE, "workspace has %zu bytes, needs %zu", workspace_bytes, skew::kFlagBytes);
  skew::DeviceInfo dev;
  if (int rc = device_info(&dev)) return rc;
  const int32_t t = hot_rows == SKEW_HOT_AUTO ? skew::materialize_max_hot_rows(dev) : hot_rows;
  const hipStream_t s = (hipStream_t)stream;
  const hipError_t e = skew::launch_materialize(fact_keys, n_fact, dim_col, n_rows, t, out, (int32_t *)workspace, dev, s);
  if (e != hipSuccess) return hip_fail(e, "materialize launch");
  if (check_enabled()) return read_flag(workspace, s);
  return ok();
}

int select_fact_rows(const int32_t *fact_keys, int64_t n_fact, const int32_t *dim_col, int32_t n_rows, int32_t lt,
                     int32_t hot_rows, int32_t *out_offsets, int64_t *out_count, void *workspace,
                     size_t workspace_bytes, void *stream) {
  if (n_fact < 0 || n_fact >= ((int64_t)1 << 31)) return fail(SKEW_EINVAL, "n_fact must be in [0, 2^31)");
  if (n_rows < 1) return fail(SKEW_EINVAL, "n_rows must be >= 1");
  if (n_fact > 0 && (!fact_keys || !out_offsets)) return fail(SKEW_EINVAL, "fact_keys and out_offsets are required");
  if (!dim_col || !out_count) return fail(SKEW_EINVAL, "dim_col and out_count are required");
  if (!workspace) return fail(SKEW_EINVAL, "workspace is NULL");
  if (hot_rows < SKEW_HOT_AUTO) return fail(SKEW_EINVAL, "hot_rows must be >= 0 or SKEW_HOT_AUTO");
  if (!aligned4(fact_keys) || !aligned4(dim_col) || !aligned4(out_offsets))
    return fail(SKEW_EINVAL, "32-bit arrays must be 4-byte aligned");
  if ((uintptr_t)out_count & 7u) return fail(SKEW_EINVAL, "out_count must be 8-byte aligned");
  if (!aligned256(workspace)) return fail(SKEW_EINVAL, "workspace must be 256-byte aligned");
  const size_t need = skew_workspace_bytes(SKEW_OP_SELECT, n_fact, n_rows);
  if (workspace_bytes < need) return fail(SKEW_ENOSPACE, "workspace has %zu bytes, needs %zu", workspace_bytes, need);
  skew::DeviceInfo dev;
  if (int rc = device_info(&dev)) return rc;
  const skew::DeviceInfo pdev = part_device(dev);
  int64_t t = hot_rows == SKEW_HOT_AUTO ? skew::select_max_hot_rows(dev) : hot_rows;
  if (t > n_rows) t = n_rows;
  const hipStream_t s = (hipStream_t)stream;
  char *ws = (char *)workspace;
  const hipError_t e = skew::launch_select(fact_keys, n_fact, dim_col, n_rows, lt, (int32_t)t, out_offsets, out_count,
                                           (int32_t *)ws, ws + skew::kFlagBytes, pdev, s);
  if (e != hipSuccess) return hip_fail(e, "select launch");
  if (check_enabled()) return read_flag(workspace, s);
  return ok();
}

int heavy_hitter_counts(const int32_t *ranked_keys, int64_t n_fact, int32_t n_keys, int32_t k, const int32_t *perm,
                        int32_t *out_keys, int64_t *out_count, void *workspace, size_t workspace_bytes,
                        void *stream) {
  if (n_fact < 0) return fail(SKEW_EINVAL, "n_fact must be >= 0");
  if (n_keys < 1) return fail(SKEW_EINVAL, "n_keys must be >= 1");
  if (k < 0 || k > n_keys) return fail(SKEW_EINVAL, "k must be in [0, n_keys]");
  if (n_fact > 0 && !ranked_keys) return fail(SKEW_EINVAL, "ranked_keys is NULL");
  if (k > 0 && (!out_keys || !out_count)) return fail(SKEW_EINVAL, "outputs are required");
  if (!workspace) return fail(SKEW_EINVAL, "workspace is NULL");
  if (!aligned4(ranked_keys) || !aligned4(perm) || !aligned4(out_keys))
    return fail(SKEW_EINVAL, "32-bit arrays must be 4-byte aligned");
  if ((uintptr_t)out_count & 7u) return fail(SKEW_EINVAL, "out_count must be 8-byte aligned");
  if (!aligned256(workspace)) return fail(SKEW_EINVAL, "workspace must be 256-byte aligned");
  if (workspace_bytes < skew::kFlagBytes)
    return fail(SKEW_ENOSPACE, "workspace has %zu bytes, needs %zu", workspace_bytes, skew::kFlagBytes);
  skew::DeviceInfo dev;
  if (int rc = device_info(&dev)) return rc;
  const hipStream_t s = (hipStream_t)stream;
  const hipError_t e =
      skew::launch_heavy(ranked_keys, n_fact, n_keys, k, perm, out_keys, out_count, (int32_t *)workspace, dev, s);
  if (e != hipSuccess) return hip_fail(e, "heavy hitter launch");
  if (check_enabled()) return read_flag(workspace, s);
  return ok();
}

int stream_probe(const void *buf, size_t bytes, uint64_t *out_sum, void *stream) {
  if (!out_sum) return fail(SKEW_EINVAL, "out_sum is NULL");
  if (bytes > 0 && !buf) return fail(SKEW_EINVAL, "buf is NULL");
  if (((uintptr_t)buf & 15u) || (bytes & 15u)) return fail(SKEW_EINVAL, "buf and bytes must be 16-byte multiples");
  if ((uintptr_t)out_sum & 7u) return fail(SKEW_EINVAL, "out_sum must be 8-byte aligned");
  skew::DeviceInfo dev;
  if (int rc = device_info(&dev)) return rc;
  const hipError_t e = skew::launch_stream_probe(buf, bytes, out_sum, dev, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "stream probe");
  return ok();
}

int cache_model_hit_rate(const uint32_t *counts_by_rank, int32_t n_keys, const int32_t *rank,
                         int32_t values_per_line, int64_t cache_lines, double *out_hit, void *workspace,
                         size_t workspace_bytes, void *stream) {
  if (n_keys < 1) return fail(SKEW_EINVAL, "n_keys must be >= 1");
  if (!counts_by_rank || !out_hit) return fail(SKEW_EINVAL, "counts_by_rank and out_hit are required");
  if (values_per_line < 1) return fail(SKEW_EINVAL, "values_per_line must be >= 1");
  if (cache_lines < 1) return fail(SKEW_EINVAL, "cache_lines must be >= 1");
  if (!workspace) return fail(SKEW_EINVAL, "workspace is NULL");
  if (!aligned4(counts_by_rank) || !aligned4(rank)) return fail(SKEW_EINVAL, "32-bit arrays must be 4-byte aligned");
  if (!aligned256(workspace)) return fail(SKEW_EINVAL, "workspace must be 256-byte aligned");
  const size_t need = skew::kFlagBytes + round_up(skew::model_workspace_bytes(n_keys, values_per_line));
  if (workspace_bytes < need) return fail(SKEW_ENOSPACE, "workspace has %zu bytes, needs %zu", workspace_bytes, need);
  skew::DeviceInfo dev;
  if (int rc = device_info(&dev)) return rc;
  const hipError_t e = skew::launch_cache_model(counts_by_rank, n_keys, rank, values_per_line, cache_lines,
                                                (char *)workspace + skew::kFlagBytes, out_hit, dev,
                                                (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "cache model");
  return ok();
}

namespace {

int star_check(const int32_t *prod_keys, const int32_t *cust_keys, const int64_t *query_start,
               const int32_t *query_cust_lt, int32_t n_queries, const int32_t *prod_price,
               const int8_t *prod_category, int32_t n_prod, const int8_t *cust_segment, int32_t n_cust,
               int64_t *out_sum, int64_t *out_count, void *workspace, size_t workspace_bytes) {
  if (n_queries < 1 || n_queries > skew::kMaxStarQueries) return fail(SKEW_EINVAL, "n_queries must be in [1, 4096]");
  if (n_prod < 1 || n_cust < 1) return fail(SKEW_EINVAL, "n_prod and n_cust must be >= 1");
  if (!prod_keys || !cust_keys || !query_start || !query_cust_lt)
    return fail(SKEW_EINVAL, "keys and the query table are required");
  if (!prod_price || !prod_category || !cust_segment) return fail(SKEW_EINVAL, "dimension columns are required");
  if (!out_sum || !out_count) return fail(SKEW_EINVAL, "outputs are required");
  if (!workspace) return fail(SKEW_EINVAL, "workspace is NULL");
  if (((uintptr_t)prod_keys & 15u) || ((uintptr_t)cust_keys & 15u))
    return fail(SKEW_EINVAL, "key columns must be 16-byte aligned");
  if (((uintptr_t)query_start & 7u) || ((uintptr_t)out_sum & 7u) || ((uintptr_t)out_count & 7u))
    return fail(SKEW_EINVAL, "64-bit arrays must be 8-byte aligned");
  if (!aligned4(query_cust_lt) || !aligned4(prod_price)) return fail(SKEW_EINVAL, "32-bit arrays must be 4-byte aligned");
  if (!aligned256(workspace)) return fail(SKEW_EINVAL, "workspace must be 256-byte aligned");
  const size_t need = skew::kFlagBytes + round_up(skew::star_workspace_bytes(n_prod, n_cust, n_queries));
  if (workspace_bytes < need) return fail(SKEW_ENOSPACE, "workspace has %zu bytes, needs %zu", workspace_bytes, need);
  return SKEW_OK;
}

// Defaults and clamps of a tuning on this device.
skew_star_tuning star_resolve(const skew_star_tuning *t, int32_t n_prod, int32_t n_cust, int32_t nq,
                              const skew::DeviceInfo &dev) {
  skew_star_tuning r;
  r.cust_hot_rows = t ? t->cust_hot_rows : 262144;
  r.tile_rows = t ? t->tile_rows : 262144;
  r.blocks = t && t->blocks > 0 ? t->blocks : dev.cu_count;
  if (r.cust_hot_rows < 0) r.cust_hot_rows = 0;
  if (r.cust_hot_rows > n_cust) r.cust_hot_rows = n_cust;
  int32_t cmax = skew::kStarMaxCustHot < n_cust ? skew::kStarMaxCustHot : n_cust;
  const int32_t cfit = skew::star_max_cust_hot(nq, dev);
  if (cmax > cfit) cmax = cfit;
  if (r.cust_hot_rows > cmax) r.cust_hot_rows = cmax;
  const int32_t pmax = skew::star_max_prod_hot(r.cust_hot_rows, nq, dev);
  r.prod_hot_rows = t && t->prod_hot_rows >= 0 ? t->prod_hot_rows : pmax;
  if (r.prod_hot_rows > pmax) r.prod_hot_rows = pmax;
  if (r.prod_hot_rows > n_prod) r.prod_hot_rows = n_prod;
  if (r.prod_hot_rows < 0) r.prod_hot_rows = 0;
  if (r.tile_rows < 1024) r.tile_rows = 1024;
  if (r.tile_rows > (1 << 24)) r.tile_rows = 1 << 24;
  return r;
}

}  // namespace

int star_join_batch(const int32_t *prod_keys, const int32_t *cust_keys, const int64_t *query_start,
                    const int32_t *query_cust_lt, int32_t n_queries, const int32_t *prod_price,
                    const int8_t *prod_category, int32_t n_prod, const int8_t *cust_segment, int32_t n_cust,
                    const skew_star_tuning *tuning, int64_t *out_sum, int64_t *out_count, void *workspace,
                    size_t workspace_bytes, void *stream) {
  if (int rc = star_check(prod_keys, cust_keys, query_start, query_cust_lt, n_queries, prod_price, prod_category,
                          n_prod, cust_segment, n_cust, out_sum, out_count, workspace, workspace_bytes))
    return rc;
  skew::DeviceInfo dev;
  if (int rc = device_info(&dev)) return rc;
  const skew_star_tuning t = star_resolve(tuning, n_prod, n_cust, n_queries, dev);
  const hipStream_t s = (hipStream_t)stream;
  const hipError_t e = skew::launch_star(prod_keys, cust_keys, query_start, query_cust_lt, n_queries, prod_price,
                                         prod_category, n_prod, cust_segment, n_cust, t.prod_hot_rows,
                                         t.cust_hot_rows, t.tile_rows, t.blocks, out_sum, out_count,
                                         (int32_t *)workspace, (char *)workspace + skew::kFlagBytes, dev, s);
  if (e != hipSuccess) return hip_fail(e, "star join launch");
  if (check_enabled()) return read_flag(workspace, s);
  return ok();
}

int star_join_autotune(const int32_t *prod_keys, const int32_t *cust_keys, const int64_t *query_start,
                       const int32_t *query_cust_lt, int32_t n_queries, const int32_t *prod_price,
                       const int8_t *prod_category, int32_t n_prod, const int8_t *cust_segment, int32_t n_cust,
                       int64_t *out_sum, int64_t *out_count, skew_star_tuning *best, float *best_ms,
                       void *workspace, size_t workspace_bytes, void *stream) {
  if (int rc = star_check(prod_keys, cust_keys, query_start, query_cust_lt, n_queries, prod_price, prod_category,
                          n_prod, cust_segment, n_cust, out_sum, out_count, workspace, workspace_bytes))
    return rc;
  if (!best || !best_ms) return fail(SKEW_EINVAL, "best and best_ms are required");
  skew::DeviceInfo dev;
  if (int rc = device_info(&dev)) return rc;
  const hipStream_t s = (hipStream_t)stream;
  constexpr int kReps = 3;  // timed runs per candidate (after one warm-up); the median counts
  hipEvent_t ev[kReps + 1] = {};
  hipError_t e = hipSuccess;
  for (int i = 0; i <= kReps && e == hipSuccess; ++i) e = hipEventCreate(&ev[i]);
  if (e != hipSuccess) {
    for (hipEvent_t x : ev)
      if (x) (void)hipEventDestroy(x);
    return hip_fail(e, "autotune events");
  }
  const int32_t cust_cand[] = {0, 65536, 262144, 524288, 786432, 1048576};
  const int32_t tile_cand[] = {65536, 262144, 1048576};
  const int32_t block_cand[] = {dev.cu_count, 2 * dev.cu_count};
  float best_t = -1.f;
  skew_star_tuning arg{-1, 0, 0, 0};
  for (int32_t tc : cust_cand) {
    for (int32_t tr : tile_cand) {
      for (int32_t nb : block_cand) {
        arg.cust_hot_rows = tc;
        arg.tile_rows = tr;
        arg.blocks = nb;
        const skew_star_tuning t = star_resolve(&arg, n_prod, n_cust, n_queries, dev);
        auto run = [&]() {
          return skew::launch_star(prod_keys, cust_keys, query_start, query_cust_lt, n_queries, prod_price,
                                   prod_category, n_prod, cust_segment, n_cust, t.prod_hot_rows, t.cust_hot_rows,
                                   t.tile_rows, t.blocks, out_sum, out_count, (int32_t *)workspace,
                                   (char *)workspace + skew::kFlagBytes, dev, s);
        };
        e = run();  // warm-up
        if (e == hipSuccess) e = hipEventRecord(ev[0], s);
        for (int i = 0; i < kReps && e == hipSuccess; ++i) {
          e = run();
          if (e == hipSuccess) e = hipEventRecord(ev[i + 1], s);
        }
        if (e == hipSuccess) e = hipEventSynchronize(ev[kReps]);
        float ms[kReps] = {};
        for (int i = 0; i < kReps && e == hipSuccess; ++i) e = hipEventElapsedTime(&ms[i], ev[i], ev[i + 1]);
        if (e != hipSuccess) break;
        std::sort(ms, ms + kReps);
        const float med = ms[kReps / 2];
        if (best_t < 0.f || med < best_t) {
          best_t = med;
          *best = t;
        }
      }
      if (e != hipSuccess) break;
    }
    if (e != hipSuccess) break;
  }
  for (hipEvent_t x : ev) (void)hipEventDestroy(x);
  if (e != hipSuccess) return hip_fail(e, "autotune");
  *best_ms = best_t;
  return ok();
}

}  // extern "C"

namespace {

// Cost model of the threshold choice.  Bytes a fact row at or above t moves in
// the partitioned forms beyond reading its own columns: the join writes its
// key to a segment (4), the scatter reads it and writes a 2-byte offset (4 + 2,
// partial lines widen the writes to about 3), pass 3 reads the offset (2); the
// group-by moves a 4-byte record four times.
constexpr double kJoinColdBytes = 13.0;
constexpr double kGroupColdBytes = 16.0;
// Fixed cost of one round of a partitioned form (plan kernels and launches,
// about 20 us), in bytes at the read rate of the device (6 TB/s).
constexpr double kRoundFixedBytes = 128.0e6;
constexpr double kLineBytes = 128.0;     // an L2 miss of a gather or an atomic moves one line
constexpr int64_t kL2Lines = 32768;      // one XCD's 4 MB L2 (each XCD sees the whole access stream)

// counts[0, n) of a device array of frequencies in rank order, added up into
// prefix[0, n] on the host (waits for the stream).
int host_prefix(const uint32_t *counts, int32_t n, std::vector<uint64_t> &prefix, hipStream_t s) {
  std::vector<uint32_t> h((size_t)n);
  hipError_t e = n > 0 ? hipMemcpyAsync(h.data(), counts, (size_t)n * 4, hipMemcpyDeviceToHost, s) : hipSuccess;
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "copying the frequencies");
  prefix.assign((size_t)n + 1, 0);
  for (int32_t i = 0; i < n; ++i) prefix[(size_t)i + 1] = prefix[(size_t)i] + h[(size_t)i];
  return SKEW_OK;
}

// Leading ranks (at most cap) whose frequency reaches `threshold` (frequencies
// do not increase along the ranks).
int32_t ranks_reaching(const std::vector<uint64_t> &prefix, int32_t cap, double threshold) {
  int32_t t = 0;
  while (t < cap && (double)(prefix[(size_t)t + 1] - prefix[(size_t)t]) >= threshold) ++t;
  return t;
}

// Modelled L2 hit rate of the lookups of ranks [t, n_keys) (Section 3.3's model, frequency-ordered lines of
// `per_line` values).
int residual_hit(const uint32_t *counts, int32_t n_keys, int32_t t, int32_t per_line, double *hit, void *ws,
                 size_t ws_bytes, const skew::DeviceInfo &dev, hipStream_t s) {
  *hit = 1.0;
  if (t >= n_keys) return SKEW_OK;
  const size_t need = skew::kFlagBytes + round_up(skew::model_workspace_bytes(n_keys - t, per_line));
  if (ws_bytes < need) return fail(SKEW_ENOSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, need);
  const hipError_t e = skew::launch_cache_model(counts + t, n_keys - t, nullptr, per_line, kL2Lines,
                                                (char *)ws + skew::kFlagBytes, hit, dev, s);
  return e == hipSuccess ? SKEW_OK : hip_fail(e, "cache model");
}

}  // namespace

extern "C" {

int skew_join_choose(const uint32_t *counts_by_rank, int32_t n_keys, int64_t n_fact, int32_t group_by_category,
                     skew_choice *out, void *workspace, size_t workspace_bytes, void *stream) {
  if (n_keys < 1 || n_fact < 0) return fail(SKEW_EINVAL, "bad sizes");
  if (!counts_by_rank || !out || !workspace) return fail(SKEW_EINVAL, "counts_by_rank, out and workspace are required");
  if (group_by_category != 0 && group_by_category != 1) return fail(SKEW_EINVAL, "group_by_category must be 0 or 1");
  if (!aligned4(counts_by_rank)) return fail(SKEW_EINVAL, "counts_by_rank must be 4-byte aligned");
  if (!aligned256(workspace)) return fail(SKEW_EINVAL, "workspace must be 256-byte aligned");
  skew::DeviceInfo dev;
  if (int rc = device_info(&dev)) return rc;
  const hipStream_t s = (hipStream_t)stream;
  const int groups = group_by_category ? 16 : 1;
  const skew::DeviceInfo pdev = part_device(dev);
  int32_t cap = skew::join_max_hot_rows(groups, dev);
  if (cap > n_keys) cap = n_keys;
  std::vector<uint64_t> prefix;
  if (int rc = host_prefix(counts_by_rank, cap, prefix, s)) return rc;
  const skew::JoinPlan pl = skew::join_plan(n_fact, n_keys, 0, groups, pdev);
  const int64_t rounds = pl.round > 0 ? (n_fact + pl.round - 1) / pl.round : 0;
  // A row earns its place in the LDS prefix when the cold bytes its keys would move exceed the bytes of
  // copying it into every workgroup of every round.
  const double stage = 4.0 * pl.blocks * (double)(rounds > 0 ? rounds : 1);
  const int32_t t = ranks_reaching(prefix, cap, stage / kJoinColdBytes);
  const double F = (double)n_fact, cold = F - (double)prefix[(size_t)t];
  double hit = 1.0;
  if (int rc = residual_hit(counts_by_rank, n_keys, t, 32, &hit, workspace, workspace_bytes, dev, s)) return rc;
  out->hot_rows = t;
  out->cold_share = F > 0 ? cold / F : 0.0;
  out->l2_hit = hit;
  // The single pass reads the keys and gathers every cold lookup (a line per L2 miss); the partitioned form
  // moves kJoinColdBytes per cold key and reads every dimension row past t once in pass 3.
  out->bytes_single = 4.0 * F + cold * (1.0 - hit) * kLineBytes + 4.0 * t * dev.cu_count;
  out->bytes_partitioned = 4.0 * F + cold * kJoinColdBytes + stage * t + 4.0 * (double)(n_keys - t) +
                           kRoundFixedBytes * (double)rounds;
  out->partitioned = n_fact >= skew::kPartitionMinFact && out->bytes_partitioned < out->bytes_single ? 1 : 0;
  return ok();
}

int skew_group_choose(const uint32_t *counts_by_rank, int32_t n_groups, int64_t n_fact, skew_choice *out,
                      void *workspace, size_t workspace_bytes, void *stream) {
  if (n_groups < 1 || n_fact < 0) return fail(SKEW_EINVAL, "bad sizes");
  if (!counts_by_rank || !out || !workspace) return fail(SKEW_EINVAL, "counts_by_rank, out and workspace are required");
  if (!aligned4(counts_by_rank)) return fail(SKEW_EINVAL, "counts_by_rank must be 4-byte aligned");
  if (!aligned256(workspace)) return fail(SKEW_EINVAL, "workspace must be 256-byte aligned");
  skew::DeviceInfo dev;
  if (int rc = device_info(&dev)) return rc;
  const hipStream_t s = (hipStream_t)stream;
  const skew::DeviceInfo pdev = part_device(dev);
  const skew::GroupPlan pl = skew::group_plan(n_fact, n_groups, pdev);
  // the launch's shared slice table: record slices and pair slices
  const int32_t Q = pl.slices + skew::group_narrow_slices(pl);
  const bool can_partition = n_fact >= skew::kPartitionMinFact && pl.slices > 0 && Q <= skew::kMaxSlices;
  int32_t cap = can_partition ? skew::group_split_max_hot_groups(Q, dev) : skew::group_max_hot_groups(dev);
  if (cap > n_groups) cap = n_groups;
  std::vector<uint64_t> prefix;
  if (int rc = host_prefix(counts_by_rank, cap, prefix, s)) return rc;
  const int64_t rounds = pl.round > 0 ? (n_fact + pl.round - 1) / pl.round : 0;
  // A group earns its LDS bin when its cold bytes exceed clearing and flushing the bin (a 16-byte sum and
  // count read, then added to the accumulators by two atomics whose lines stay in L2) in every workgroup of
  // every round.
  const double stage = 32.0 * pl.blocks * (double)(rounds > 0 ? rounds : 1);
  const int32_t t = ranks_reaching(prefix, cap, stage / kGroupColdBytes);
  const double F = (double)n_fact, cold = F - (double)prefix[(size_t)t];
  double hit = 1.0;
  // the cold rows' atomics go to int64 sum and count words: 16 groups per 128-byte line
  if (int rc = residual_hit(counts_by_rank, n_groups, t, 16, &hit, workspace, workspace_bytes, dev, s)) return rc;
  out->hot_rows = t;
  out->cold_share = F > 0 ? cold / F : 0.0;
  out->l2_hit = hit;
  out->bytes_single = 8.0 * F + cold * (1.0 - hit) * 2.0 * kLineBytes + stage * t / (double)(rounds > 0 ? rounds : 1);
  out->bytes_partitioned = 8.0 * F + cold * kGroupColdBytes + stage * t + 16.0 * n_groups +
                           kRoundFixedBytes * (double)rounds;
  out->partitioned = can_partition && out->bytes_partitioned < out->bytes_single ? 1 : 0;
  return ok();
}

int skew_query_status(const void *workspace, size_t workspace_bytes, void *stream) {
  if (!workspace || workspace_bytes < skew::kFlagBytes) return fail(SKEW_EINVAL, "workspace is NULL or too small");
  return read_flag(workspace, (hipStream_t)stream);
}

void skew_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_on = on != 0;
}

int skew_profile_report(char *names, int names_bytes, float *ms, int *calls, int max_stages) {
  std::vector<StageRecord> recs;
  {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    recs.swap(g_prof);
  }
  std::vector<std::string> keys;
  std::vector<float> tot;
  std::vector<int> cnt;
  for (auto &r : recs) {
    float v = 0.f;
    if (hipEventSynchronize(r.stop) == hipSuccess && hipEventElapsedTime(&v, r.start, r.stop) == hipSuccess) {
      size_t i = 0;
      while (i < keys.size() && keys[i] != r.name) ++i;
      if (i == keys.size()) {
        keys.emplace_back(r.name);
        tot.push_back(0.f);
        cnt.push_back(0);
      }
      tot[i] += v;
      cnt[i] += 1;
    }
    (void)hipEventDestroy(r.start);
    (void)hipEventDestroy(r.stop);
  }
  const int n = (int)keys.size() < max_stages ? (int)keys.size() : max_stages;
  int off = 0;
  for (int i = 0; i < n; ++i) {
    if (ms) ms[i] = tot[i];
    if (calls) calls[i] = cnt[i];
    if (names && off + (int)keys[i].size() + 1 < names_bytes) {
      std::memcpy(names + off, keys[i].c_str(), keys[i].size() + 1);
      off += (int)keys[i].size() + 1;
    }
  }
  if (names && off < names_bytes) names[off] = 0;
  return n;
}

int32_t skew_max_hot_rows(int32_t group_by_category) {
  skew::DeviceInfo dev;
  if (int rc = device_info(&dev)) return rc;
  return skew::join_max_hot_rows(group_by_category ? 16 : 1, dev);
}

int32_t skew_join_hot_rows(int64_t n_fact, int32_t n_rows, int32_t group_by_category, int32_t hot_rows,
                           size_t workspace_bytes) {
  if (n_fact < 0 || n_rows < 1 || hot_rows < SKEW_HOT_AUTO || (group_by_category != 0 && group_by_category != 1))
    return fail(SKEW_EINVAL, "bad sizes or hot_rows");
  skew::DeviceInfo dev;
  if (int rc = device_info(&dev)) return rc;
  const size_t need = join_ws(n_rows);
  bool partitioned = false;
  return skew::join_hot_rows_used(n_fact, n_rows, group_by_category, hot_rows,
                                  workspace_bytes > need ? workspace_bytes - need : 0, part_device(dev), &partitioned);
}

int32_t skew_max_hot_groups(void) {
  skew::DeviceInfo dev;
  if (int rc = device_info(&dev)) return rc;
  return skew::group_split_max_hot_groups(skew::kMaxSlices, dev);
}

int64_t skew_max_hot(int op) {
  skew::DeviceInfo dev;
  if (int rc = device_info(&dev)) return rc;
  switch (op) {
    case SKEW_OP_MATERIALIZE:
      return skew::materialize_max_hot_rows(dev);
    case SKEW_OP_SELECT:
      return skew::select_max_hot_rows(dev);
    case SKEW_OP_HEAVY:
      return skew::heavy_max_lds_ranks(dev);
    case SKEW_OP_GROUP_SINGLE_PASS:
      return skew::group_max_hot_groups(dev);
    default:
      return fail(SKEW_EINVAL, "op %d has no hot prefix of its own", op);
  }
}

}  // extern "C"

// Batched evaluation: many independent systems in one persistent launch, optionally replayed
// from a HIP graph, with a launch shape chosen by timing (spline_batch_autotune).
//
// A plan holds, in device memory it owns, one EvalArgs per item (sorted by decreasing work per
// tile), the exclusive prefix of tiles per item and the work counter.  A launch is two kernels
// on one stream: k_batch_reset (zeroes the counter, so no memset node is needed in a graph) and
// k_eval_batch (the persistent kernel, one workgroup per resident slot of the GPU).
//
// Sorted plans (spline_batch_plan_sort) first put every item's points in locality order, as the
// single-system sorted call does: one counting sort over all items at once.  Item j owns the
// global buckets [bucket_base_j, bucket_base_j + buckets_j), cells grouped 2^shift per axis and
// numbered along a Morton curve (at most 2^15 per item, plus one for non-finite points), so the
// slots of its points form the contiguous range [point_start_j, point_start_j + n_pts_j) of the
// permutation, which holds item-local indices.  The kernels: clear the counts, count (each point
// finds its item by binary search), exclusive scan, scatter; then the persistent launch reads each
// item's slice of the permutation.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <numeric>
#include <vector>

#include "internal.hpp"

namespace pws {

__global__ __launch_bounds__(256) void k_fill_zero_i32(int32_t* x, int32_t n);

struct SortItem {
  Geom g;
  const double* pos;
  int32_t n_pts;
  int32_t shift;        // cells per bucket along an axis: 2^shift
  int32_t bucket_base;  // first global bucket of the item
  int32_t sentinel;     // the item's bucket of points with non-finite coordinates (its last)
  int32_t point_start;  // first slot of the item in the permutation
};

__device__ __forceinline__ int sort_item_of(const SortItem* items, int n_items, int p) {
  int lo = 0, hi = n_items - 1;                      // last item whose first slot <= p
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (items[mid].point_start <= p) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(256) void k_batch_bucket_count(const SortItem* items, int32_t n_items, int32_t n_total,
                                                            int32_t* bucket, int32_t* counts) {
  const int p = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (p >= n_total) return;
  const SortItem& it = items[sort_item_of(items, n_items, p)];
  const int q = p - it.point_start;
  int i0[3];
  double t[3];
  const bool ok = reduce_point(it.g, it.pos[3 * (int64_t)q], it.pos[3 * (int64_t)q + 1], it.pos[3 * (int64_t)q + 2],
                               i0, t);
  const int32_t b = ok ? it.bucket_base + (int32_t)((spread3((uint32_t)(i0[0] >> it.shift)) << 2) |
                                                    (spread3((uint32_t)(i0[1] >> it.shift)) << 1) |
                                                    spread3((uint32_t)(i0[2] >> it.shift)))
                       : it.sentinel;
  bucket[p] = b;
  atomicAdd(&counts[b], 1);
}

__global__ __launch_bounds__(256) void k_batch_bucket_scatter(const SortItem* items, int32_t n_items, int32_t n_total,
                                                              const int32_t* bucket, int32_t* offsets, int32_t* perm) {
  const int p = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (p >= n_total) return;
  const SortItem& it = items[sort_item_of(items, n_items, p)];
  perm[atomicAdd(&offsets[bucket[p]], 1)] = p - it.point_start;
}

// Zero the work counter with an ordinary vector store (a kernel node, so a captured graph holds
// no memset node).
__global__ void k_batch_reset(int32_t* counter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0;
}

struct Plan {
  int dtype = 0;
  int mode = MODE_VGL;
  int32_t tile[2] = {0, 0};           // the common shape; tile[0] = 0: per-item lanes (lanes[])
  std::vector<int32_t> lanes;         // lanes per point of each item (sorted order)
  std::vector<int> order;             // sorted position -> caller's item index
  std::vector<spl_desc> descs;        // copies of the items' descriptors (sorted order)
  std::vector<spl_item> items;        // caller's items (sorted order)
  std::vector<EvalArgs> args;         // per-item kernel arguments for the current tile
  std::vector<int32_t> tile_start;    // prefix of tiles per item for the current tile
  EvalArgs* d_items = nullptr;
  int32_t* d_tile_start = nullptr;
  int32_t* d_counter = nullptr;
  int32_t n_tiles = 0;
  int64_t n_evals = 0;
  int grid = 0;
  BatchKernel kernel = nullptr;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // sorted plans
  bool sort_on = false;
  SortItem* d_sort = nullptr;
  int32_t* d_bucket = nullptr;
  int32_t* d_counts = nullptr;
  int32_t* d_offsets = nullptr;
  int32_t* d_perm = nullptr;
  void* d_scan_temp = nullptr;
  size_t scan_temp_bytes = 0;
  int32_t n_points = 0;
  int32_t n_buckets = 0;
  std::vector<int32_t> point_start;
};

static BatchKernel pick_batch(int dtype, int mode, int g, int opl) {
  if (dtype == SPL_F64) return pick_batch_f64(mode, g, opl);
  if (dtype == SPL_F32) return pick_batch_f32(mode, g, opl);
  return pick_batch_bf16(mode, g, opl);
}

static void drop_graph(Plan* pl) {
  if (pl->exec) hipGraphExecDestroy(pl->exec);
  if (pl->graph) hipGraphDestroy(pl->graph);
  pl->exec = nullptr;
  pl->graph = nullptr;
}

// (Re)derive kernel arguments, the tile prefix and the launch grid, and upload them: with
// tile[0] > 0 every item takes the shape `tile`; with tile[0] == 0 item j (sorted order) takes
// lanes[j] lanes per point and tile[1] orbitals per lane.  Synchronous on `stream`.
static int plan_set_shapes(Plan* pl, const int32_t tile[2], const int32_t* lanes, hipStream_t stream) {
  const int n = (int)pl->items.size();
  const bool multi = tile[0] == 0;
  for (int j = 0; j < (multi ? n : 1); ++j) {
    const int32_t t[2] = {multi ? lanes[j] : tile[0], tile[1]};
    if (!tile_valid(pl->dtype, t) || t[0] < 8)
      return fail(SPL_EINVAL, "invalid batch tile (%d, %d): lanes per point must be 8..256", t[0], t[1]);
  }
  BatchKernel k = pick_batch(pl->dtype, pl->mode, multi ? 0 : tile[0], tile[1]);
  if (!k) return fail(SPL_EINVAL, "invalid batch tile (%d, %d)", tile[0], tile[1]);
  pl->args.resize(n);
  pl->tile_start.assign(n + 1, 0);
  pl->lanes.resize(n);
  int64_t tiles = 0;
  for (int j = 0; j < n; ++j) {
    const spl_item& it = pl->items[j];
    pl->lanes[j] = multi ? lanes[j] : tile[0];
    const int per_tile = 256 / pl->lanes[j];
    fill_eval_args(&pl->descs[j], it.table, it.n_pts, it.pos, it.v, it.grad, it.lap, 0, tile[1], &pl->args[j]);
    pl->args[j].lanes = pl->lanes[j];
    if (pl->sort_on) pl->args[j].perm = pl->d_perm + pl->point_start[j];
    pl->tile_start[j] = (int32_t)tiles;
    tiles += (it.n_pts + per_tile - 1) / per_tile;
  }
  if (tiles > 0x7fffffffLL) return fail(SPL_EINVAL, "batch has too many tiles");
  pl->tile_start[n] = (int32_t)tiles;
  pl->n_tiles = (int32_t)tiles;
  int rc;
  if ((rc = hip_fail(hipMemcpyAsync(pl->d_items, pl->args.data(), sizeof(EvalArgs) * n, hipMemcpyHostToDevice, stream),
                     "upload batch items")))
    return rc;
  if ((rc = hip_fail(hipMemcpyAsync(pl->d_tile_start, pl->tile_start.data(), sizeof(int32_t) * (n + 1),
                                    hipMemcpyHostToDevice, stream), "upload batch tiles")))
    return rc;
  if ((rc = hip_fail(hipStreamSynchronize(stream), "hipStreamSynchronize"))) return rc;
  int dev = 0, cus = 0, per_cu = 0;
  if ((rc = hip_fail(hipGetDevice(&dev), "hipGetDevice"))) return rc;
  if ((rc = hip_fail(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "device attribute")))
    return rc;
  if ((rc = hip_fail(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(k), 256, 0),
                     "occupancy query")))
    return rc;
  const int64_t slots = (int64_t)std::max(1, cus) * std::max(1, per_cu);
  pl->grid = (int)std::max<int64_t>(1, std::min<int64_t>(slots, tiles));
  pl->kernel = k;
  pl->tile[0] = tile[0];
  pl->tile[1] = tile[1];
  drop_graph(pl);
  return SPL_OK;
}

static int plan_set_tile(Plan* pl, const int32_t tile[2], hipStream_t stream) {
  if (tile[0] == 0) return fail(SPL_EINVAL, "invalid batch tile (0, %d): lanes per point must be 8..256", tile[1]);
  return plan_set_shapes(pl, tile, nullptr, stream);
}

static int plan_launch(Plan* pl, hipStream_t stream) {
  if (pl->n_tiles == 0) return SPL_OK;
  int rc;
  if (pl->sort_on) {
    const int n_items = (int)pl->items.size();
    const unsigned pb = (unsigned)((pl->n_points + 255) / 256);
    hipLaunchKernelGGL(k_fill_zero_i32, dim3((unsigned)std::min(1024, (pl->n_buckets + 255) / 256)), dim3(256), 0,
                       stream, pl->d_counts, pl->n_buckets);
    if ((rc = hip_fail(hipGetLastError(), "bucket clear launch"))) return rc;
    hipLaunchKernelGGL(k_batch_bucket_count, dim3(pb), dim3(256), 0, stream, pl->d_sort, (int32_t)n_items,
                       pl->n_points, pl->d_bucket, pl->d_counts);
    if ((rc = hip_fail(hipGetLastError(), "bucket count launch"))) return rc;
    size_t tb = pl->scan_temp_bytes;
    if ((rc = hip_fail(hipcub::DeviceScan::ExclusiveSum(pl->d_scan_temp, tb, pl->d_counts, pl->d_offsets,
                                                        pl->n_buckets, stream),
                       "bucket scan")))
      return rc;
    hipLaunchKernelGGL(k_batch_bucket_scatter, dim3(pb), dim3(256), 0, stream, pl->d_sort, (int32_t)n_items,
                       pl->n_points, pl->d_bucket, pl->d_offsets, pl->d_perm);
    if ((rc = hip_fail(hipGetLastError(), "bucket scatter launch"))) return rc;
  }
  hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, stream, pl->d_counter);
  rc = hip_fail(hipGetLastError(), "batch counter reset launch");
  if (rc) return rc;
  BatchArgs b;
  b.items = pl->d_items;
  b.tile_start = pl->d_tile_start;
  b.counter = pl->d_counter;
  b.n_items = (int32_t)pl->items.size();
  b.n_tiles = pl->n_tiles;
  hipLaunchKernelGGL(pl->kernel, dim3(pl->grid), dim3(256), 0, stream, b);
  return hip_fail(hipGetLastError(), "batch launch");
}

// Median of three timed launches (after one untimed), ms.
static int time_plan(Plan* pl, hipStream_t s, hipEvent_t e0, hipEvent_t e1, float* ms) {
  int rc = plan_launch(pl, s);
  float times[3];
  for (int r = 0; r < 3 && !rc; ++r) {
    hipEventRecord(e0, s);
    rc = plan_launch(pl, s);
    hipEventRecord(e1, s);
    if (!rc) rc = hip_fail(hipEventSynchronize(e1), "hipEventSynchronize");
    if (!rc) rc = hip_fail(hipEventElapsedTime(&times[r], e0, e1), "hipEventElapsedTime");
  }
  if (rc) return rc;
  std::sort(times, times + 3);
  *ms = times[1];
  return SPL_OK;
}

static void plan_free(Plan* pl) {
  if (!pl) return;
  hipDeviceSynchronize();
  drop_graph(pl);
  if (pl->cap_stream) hipStreamDestroy(pl->cap_stream);
  if (pl->d_items) hipFree(pl->d_items);
  if (pl->d_tile_start) hipFree(pl->d_tile_start);
  if (pl->d_counter) hipFree(pl->d_counter);
  for (void* p : {(void*)pl->d_sort, (void*)pl->d_bucket, (void*)pl->d_counts, (void*)pl->d_offsets,
                  (void*)pl->d_perm, pl->d_scan_temp})
    if (p) hipFree(p);
  delete pl;
}

// Allocate and fill the sorting state of a plan (once).
static int plan_sort_setup(Plan* pl, hipStream_t stream) {
  if (pl->d_sort) return SPL_OK;
  const int n = (int)pl->items.size();
  std::vector<SortItem> si(n);
  pl->point_start.assign(n, 0);
  int64_t pts = 0, buckets = 0;
  for (int j = 0; j < n; ++j) {
    const spl_desc& d = pl->descs[j];
    const int nmax = std::max(d.grid[0], std::max(d.grid[1], d.grid[2]));
    int b = 1;
    while ((1 << b) < nmax) ++b;
    const int shift = b > 5 ? b - 5 : 0;
    si[j].g = make_geom(&d);
    si[j].pos = pl->items[j].pos;
    si[j].n_pts = (int32_t)pl->items[j].n_pts;
    si[j].shift = shift;
    si[j].bucket_base = (int32_t)buckets;
    buckets += (int64_t)1 << (3 * (b - shift));
    si[j].sentinel = (int32_t)buckets;
    buckets += 1;
    si[j].point_start = (int32_t)pts;
    pl->point_start[j] = (int32_t)pts;
    pts += pl->items[j].n_pts;
  }
  if (pts > 0x7fffffffLL || buckets > 0x7fffffffLL) return fail(SPL_EINVAL, "batch too large to sort");
  pl->n_points = (int32_t)pts;
  pl->n_buckets = (int32_t)buckets;
  int rc = hip_fail(hipcub::DeviceScan::ExclusiveSum(nullptr, pl->scan_temp_bytes, (const int32_t*)nullptr,
                                                     (int32_t*)nullptr, pl->n_buckets, stream),
                    "scan size query");
  if (rc) return rc;
  const size_t np = (size_t)std::max<int64_t>(pts, 1), nb = (size_t)buckets;
  if (hipMalloc(&pl->d_sort, sizeof(SortItem) * n) != hipSuccess || hipMalloc(&pl->d_bucket, 4 * np) != hipSuccess ||
      hipMalloc(&pl->d_counts, 4 * nb) != hipSuccess || hipMalloc(&pl->d_offsets, 4 * nb) != hipSuccess ||
      hipMalloc(&pl->d_perm, 4 * np) != hipSuccess ||
      hipMalloc(&pl->d_scan_temp, std::max<size_t>(pl->scan_temp_bytes, 1)) != hipSuccess)
    return fail(SPL_ENOMEM, "sorted batch: device allocation failed");
  if ((rc = hip_fail(hipMemcpyAsync(pl->d_sort, si.data(), sizeof(SortItem) * n, hipMemcpyHostToDevice, stream),
                     "upload sort items")))
    return rc;
  return hip_fail(hipStreamSynchronize(stream), "hipStreamSynchronize");
}

}  // namespace pws

using namespace pws;

extern "C" {

int spline_batch_plan_create(const spl_item* items, int32_t n_items, const int32_t* tile, void* stream,
                             void** plan_out) {
  clear_error();
  if (!items || !plan_out) return fail(SPL_EINVAL, "items and plan must be non-NULL");
  if (n_items < 1) return fail(SPL_EINVAL, "n_items = %d < 1", n_items);
  *plan_out = nullptr;
  int rc;
  for (int j = 0; j < n_items; ++j) {
    const spl_item& it = items[j];
    if (!it.d) return fail(SPL_EINVAL, "item %d has no descriptor", j);
    if ((rc = check_eval_args(it.d, it.table, it.n_pts, it.pos))) return fail(rc, "item %d: %s", j, spline_last_error());
    if (it.n_pts > 0 && (rc = check_vgl_outputs(it.d, it.v, it.grad, it.lap)))
      return fail(rc, "item %d: %s", j, spline_last_error());
    if (it.d->basis != SPL_BSPLINE || it.d->sep_grad || it.d->bloch)
      return fail(SPL_EUNSUPPORTED, "item %d: batched plans take real B-spline tables without separate gradients", j);
    if (it.d->dtype != items[0].d->dtype || it.d->has_lap != items[0].d->has_lap)
      return fail(SPL_EINVAL, "item %d: all items of a plan must share dtype and has_lap", j);
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  Plan* pl = new Plan();
  pl->dtype = items[0].d->dtype;
  pl->mode = items[0].d->has_lap ? MODE_VGL_SEPLAP : MODE_VGL;
  // order: most work per tile first (orbitals per point), so the tail of the launch is short tiles
  std::vector<int> order(n_items);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return items[a].d->o_pad > items[b].d->o_pad; });
  int best = 0;
  pl->order = order;
  for (int j : order) {
    pl->descs.push_back(*items[j].d);
    pl->items.push_back(items[j]);
    pl->n_evals += items[j].n_pts * (int64_t)items[j].d->n_orb;
  }
  for (int j = 0; j < n_items; ++j)
    if (pl->items[j].n_pts * (int64_t)pl->descs[j].o_pad > pl->items[best].n_pts * (int64_t)pl->descs[best].o_pad)
      best = j;
  for (auto& it : pl->items) it.d = nullptr;     // descriptors live in pl->descs
  if ((rc = hip_fail(hipMalloc(&pl->d_items, sizeof(EvalArgs) * n_items), "hipMalloc")) ||
      (rc = hip_fail(hipMalloc(&pl->d_tile_start, sizeof(int32_t) * (n_items + 1)), "hipMalloc")) ||
      (rc = hip_fail(hipMalloc(&pl->d_counter, sizeof(int32_t)), "hipMalloc"))) {
    plan_free(pl);
    return rc == SPL_EHIP ? fail(SPL_ENOMEM, "batch plan allocation failed") : rc;
  }
  int32_t t[2];
  if (tile) {
    t[0] = tile[0];
    t[1] = tile[1];
  } else {
    tile_for(&pl->descs[best], t);              // the heaviest item's tuned (or default) shape
    if (t[0] < 8) t[0] = 8;
  }
  if ((rc = plan_set_tile(pl, t, s))) {
    plan_free(pl);
    return rc;
  }
  *plan_out = pl;
  return SPL_OK;
}

int spline_batch_eval_vgl(void* plan, void* stream) {
  clear_error();
  if (!plan) return fail(SPL_EINVAL, "plan is NULL");
  return plan_launch(static_cast<Plan*>(plan), static_cast<hipStream_t>(stream));
}

int spline_batch_graph_launch(void* plan, void* stream) {
  clear_error();
  if (!plan) return fail(SPL_EINVAL, "plan is NULL");
  Plan* pl = static_cast<Plan*>(plan);
  int rc;
  if (!pl->exec) {
    if (!pl->cap_stream &&
        (rc = hip_fail(hipStreamCreateWithFlags(&pl->cap_stream, hipStreamNonBlocking), "hipStreamCreate")))
      return rc;
    if ((rc = hip_fail(hipStreamBeginCapture(pl->cap_stream, hipStreamCaptureModeThreadLocal), "begin capture")))
      return rc;
    rc = plan_launch(pl, pl->cap_stream);
    hipGraph_t g = nullptr;
    const int rc2 = hip_fail(hipStreamEndCapture(pl->cap_stream, &g), "end capture");
    if (rc || rc2) {
      if (g) hipGraphDestroy(g);
      return rc ? rc : rc2;
    }
    pl->graph = g;
    if ((rc = hip_fail(hipGraphInstantiate(&pl->exec, pl->graph, nullptr, nullptr, 0), "graph instantiate"))) {
      drop_graph(pl);
      return rc;
    }
  }
  return hip_fail(hipGraphLaunch(pl->exec, static_cast<hipStream_t>(stream)), "graph launch");
}

int spline_batch_autotune(void* plan, void* stream, int32_t tile_out[2]) {
  clear_error();
  if (!plan || !tile_out) return fail(SPL_EINVAL, "plan and tile_out must be non-NULL");
  Plan* pl = static_cast<Plan*>(plan);
  hipStream_t s = static_cast<hipStream_t>(stream);
  int set[3];
  opl_set(pl->dtype, set);
  hipEvent_t e0, e1;
  int rc;
  if ((rc = hip_fail(hipEventCreate(&e0), "hipEventCreate"))) return rc;
  if ((rc = hip_fail(hipEventCreate(&e1), "hipEventCreate"))) {
    hipEventDestroy(e0);
    return rc;
  }
  const int n = (int)pl->items.size();
  float best = 1e30f;
  int32_t best_tile[2] = {pl->tile[0], pl->tile[1]};
  std::vector<int32_t> best_lanes;
  // one shape for every item
  for (int k = 0; k < 3 && !rc; ++k) {
    if (k > 0 && set[k] == set[k - 1]) continue;
    for (int g = 8; g <= 256 && !rc; g <<= 1) {
      const int32_t t[2] = {g, set[k]};
      float ms = 0.f;
      if ((rc = plan_set_tile(pl, t, s)) || (rc = time_plan(pl, s, e0, e1, &ms))) break;
      if (ms < best) {
        best = ms;
        best_tile[0] = t[0];
        best_tile[1] = t[1];
      }
    }
  }
  // per item: at each orbitals-per-lane choice, the lanes per point that run the item fastest on its
  // own (the single-system kernel on the item's buffers); then the whole launch with those shapes
  for (int k = 0; k < 3 && !rc; ++k) {
    if (k > 0 && set[k] == set[k - 1]) continue;
    std::vector<int32_t> lanes(n, 8);
    for (int j = 0; j < n && !rc; ++j) {
      const spl_item& it = pl->items[j];
      if (it.n_pts == 0) continue;
      float bj = 1e30f;
      for (int g = 8; g <= 256 && !rc; g <<= 1) {
        const int32_t t[2] = {g, set[k]};
        if (!tile_valid_for(&pl->descs[j], t)) continue;
        rc = launch_eval(&pl->descs[j], it.table, it.n_pts, it.pos, it.v, it.grad, it.lap, 0, t, s);
        float times[3];
        for (int r = 0; r < 3 && !rc; ++r) {
          hipEventRecord(e0, s);
          rc = launch_eval(&pl->descs[j], it.table, it.n_pts, it.pos, it.v, it.grad, it.lap, 0, t, s);
          hipEventRecord(e1, s);
          if (!rc) rc = hip_fail(hipEventSynchronize(e1), "hipEventSynchronize");
          if (!rc) rc = hip_fail(hipEventElapsedTime(&times[r], e0, e1), "hipEventElapsedTime");
        }
        if (rc) break;
        std::sort(times, times + 3);
        if (times[1] < bj) {
          bj = times[1];
          lanes[j] = g;
        }
      }
    }
    if (rc) break;
    const int32_t t[2] = {0, set[k]};
    float ms = 0.f;
    if ((rc = plan_set_shapes(pl, t, lanes.data(), s)) || (rc = time_plan(pl, s, e0, e1, &ms))) break;
    if (ms < best) {
      best = ms;
      best_tile[0] = 0;
      best_tile[1] = set[k];
      best_lanes = lanes;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc) return rc;
  if ((rc = plan_set_shapes(pl, best_tile, best_lanes.empty() ? nullptr : best_lanes.data(), s))) return rc;
  tile_out[0] = best_tile[0];
  tile_out[1] = best_tile[1];
  return SPL_OK;
}

int spline_batch_plan_get_tiles(void* plan, int32_t* tiles_out) {
  clear_error();
  if (!plan || !tiles_out) return fail(SPL_EINVAL, "plan and tiles_out must be non-NULL");
  Plan* pl = static_cast<Plan*>(plan);
  for (size_t j = 0; j < pl->items.size(); ++j) {
    tiles_out[2 * pl->order[j]] = pl->lanes[j];
    tiles_out[2 * pl->order[j] + 1] = pl->tile[1];
  }
  return SPL_OK;
}

int spline_batch_plan_set_tiles(void* plan, const int32_t* tiles, void* stream) {
  clear_error();
  if (!plan || !tiles) return fail(SPL_EINVAL, "plan and tiles must be non-NULL");
  Plan* pl = static_cast<Plan*>(plan);
  const int n = (int)pl->items.size();
  std::vector<int32_t> lanes(n);
  for (int j = 0; j < n; ++j) {
    const int c = pl->order[j];
    if (tiles[2 * c + 1] != tiles[1])
      return fail(SPL_EINVAL, "item %d: every item of a plan takes the same orbitals per lane (%d, not %d)", c, tiles[1],
                  tiles[2 * c + 1]);
    lanes[j] = tiles[2 * c];
  }
  const int32_t t[2] = {0, tiles[1]};
  return plan_set_shapes(pl, t, lanes.data(), static_cast<hipStream_t>(stream));
}

void spline_batch_plan_destroy(void* plan) { plan_free(static_cast<Plan*>(plan)); }

int spline_batch_plan_sort(void* plan, int32_t enable, void* stream) {
  clear_error();
  if (!plan) return fail(SPL_EINVAL, "plan is NULL");
  if (enable != 0 && enable != 1) return fail(SPL_EINVAL, "enable must be 0 or 1");
  Plan* pl = static_cast<Plan*>(plan);
  hipStream_t s = static_cast<hipStream_t>(stream);
  int rc;
  if (enable && (rc = plan_sort_setup(pl, s))) return rc;
  pl->sort_on = enable != 0;
  const int32_t t[2] = {pl->tile[0], pl->tile[1]};
  const std::vector<int32_t> lanes = pl->lanes;
  return plan_set_shapes(pl, t, lanes.data(), s);   // refreshes the items' permutation pointers, drops the graph
}

int spline_batch_plan_info(void* plan, int64_t* n_tiles, int64_t* n_evals) {
  clear_error();
  if (!plan) return fail(SPL_EINVAL, "plan is NULL");
  Plan* pl = static_cast<Plan*>(plan);
  if (n_tiles) *n_tiles = pl->n_tiles;
  if (n_evals) *n_evals = pl->n_evals;
  return SPL_OK;
}

}  // extern "C"

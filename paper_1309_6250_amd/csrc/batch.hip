// Batched evaluation: many independent systems in one persistent launch, optionally replayed
// from a HIP graph, with a launch shape chosen by timing (spline_batch_autotune).
//
// A plan holds, in device memory it owns, one EvalArgs per item (sorted by decreasing work per
// tile), the exclusive prefix of tiles per item and the work counter.  A launch is two kernels
// on one stream: k_batch_reset (zeroes the counter, so no memset node is needed in a graph) and
// k_eval_batch (the persistent kernel, one workgroup per resident slot of the GPU).
#include <algorithm>
#include <numeric>
#include <vector>

#include "internal.hpp"

namespace pws {

// Zero the work counter with an ordinary vector store (a kernel node, so a captured graph holds
// no memset node).
__global__ void k_batch_reset(int32_t* counter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0;
}

struct Plan {
  int dtype = 0;
  int mode = MODE_VGL;
  int32_t tile[2] = {0, 0};
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

// (Re)derive kernel arguments, the tile prefix and the launch grid for tile shape `tile`, and
// upload them.  Synchronous on `stream`.
static int plan_set_tile(Plan* pl, const int32_t tile[2], hipStream_t stream) {
  if (!tile_valid(pl->dtype, tile) || tile[0] < 8)
    return fail(SPL_EINVAL, "invalid batch tile (%d, %d): lanes per point must be 8..256", tile[0], tile[1]);
  BatchKernel k = pick_batch(pl->dtype, pl->mode, tile[0], tile[1]);
  if (!k) return fail(SPL_EINVAL, "invalid batch tile (%d, %d)", tile[0], tile[1]);
  const int n = (int)pl->items.size();
  const int per_tile = 256 / tile[0];
  pl->args.resize(n);
  pl->tile_start.assign(n + 1, 0);
  int64_t tiles = 0;
  for (int j = 0; j < n; ++j) {
    const spl_item& it = pl->items[j];
    fill_eval_args(&pl->descs[j], it.table, it.n_pts, it.pos, it.v, it.grad, it.lap, 0, tile[1], &pl->args[j]);
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

static int plan_launch(Plan* pl, hipStream_t stream) {
  if (pl->n_tiles == 0) return SPL_OK;
  hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, stream, pl->d_counter);
  int rc = hip_fail(hipGetLastError(), "batch counter reset launch");
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

static void plan_free(Plan* pl) {
  if (!pl) return;
  hipDeviceSynchronize();
  drop_graph(pl);
  if (pl->cap_stream) hipStreamDestroy(pl->cap_stream);
  if (pl->d_items) hipFree(pl->d_items);
  if (pl->d_tile_start) hipFree(pl->d_tile_start);
  if (pl->d_counter) hipFree(pl->d_counter);
  delete pl;
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
  float best = 1e30f;
  int32_t best_tile[2] = {pl->tile[0], pl->tile[1]};
  for (int k = 0; k < 3 && !rc; ++k) {
    if (k > 0 && set[k] == set[k - 1]) continue;
    for (int g = 8; g <= 256 && !rc; g <<= 1) {
      const int32_t t[2] = {g, set[k]};
      if ((rc = plan_set_tile(pl, t, s))) break;
      if ((rc = plan_launch(pl, s))) break;       // warm-up
      float times[3];
      for (int r = 0; r < 3 && !rc; ++r) {
        hipEventRecord(e0, s);
        rc = plan_launch(pl, s);
        hipEventRecord(e1, s);
        if (!rc) rc = hip_fail(hipEventSynchronize(e1), "hipEventSynchronize");
        if (!rc) rc = hip_fail(hipEventElapsedTime(&times[r], e0, e1), "hipEventElapsedTime");
      }
      if (rc) break;
      std::sort(times, times + 3);
      if (times[1] < best) {
        best = times[1];
        best_tile[0] = t[0];
        best_tile[1] = t[1];
      }
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc) return rc;
  if ((rc = plan_set_tile(pl, best_tile, s))) return rc;
  tile_out[0] = best_tile[0];
  tile_out[1] = best_tile[1];
  return SPL_OK;
}

void spline_batch_plan_destroy(void* plan) { plan_free(static_cast<Plan*>(plan)); }

int spline_batch_plan_info(void* plan, int64_t* n_tiles, int64_t* n_evals) {
  clear_error();
  if (!plan) return fail(SPL_EINVAL, "plan is NULL");
  Plan* pl = static_cast<Plan*>(plan);
  if (n_tiles) *n_tiles = pl->n_tiles;
  if (n_evals) *n_evals = pl->n_evals;
  return SPL_OK;
}

}  // extern "C"

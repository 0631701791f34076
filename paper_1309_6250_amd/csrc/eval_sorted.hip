// spline_eval_vgl_sorted: locality-ordered forward evaluation.
//
// Points arrive in any order (walkers x electrons, spread over the whole cell), so consecutive
// points rarely share table rows and every block is gathered from memory.  On average a row of the
// table belongs to the blocks of several points (64 P / N1 N2 N3 of them), so evaluating the points
// in the order of a space-filling curve over the grid cells lets the points that one workgroup,
// and one XCD, handle in sequence find most rows of their blocks already in L2 or the Infinity
// Cache.  Steps: a counting sort of the points into buckets of cells numbered along a Morton curve
// (clear, count with atomics, exclusive scan, scatter), then the forward kernel of the descriptor's
// representation through the resulting permutation, with each XCD on a contiguous stretch of it.
// Each point's outputs go to its own row, in the caller's order, with the arithmetic of the unsorted
// launch: bitwise the same results.
#include <hipcub/hipcub.hpp>

#include <mutex>

#include "internal.hpp"

namespace pws {

EvalKernel eval_kernel_for(const spl_desc* d, int values_only, const int32_t tile[2], int cached);

// Buckets: cells grouped 2^shift per axis and numbered along the Morton curve (3 x `bits` bits, at most
// 18), so the bucket index space has at most 2^18 entries; points with non-finite coordinates go to
// the extra last bucket.  A counting sort into buckets gives the locality order; the order inside a
// bucket is whatever the scatter's atomics produce, which changes no output (every point's arithmetic
// is independent of the lane and workgroup that run it).
struct BucketGeom {
  int bits;     // bits per axis of a bucket coordinate
  int shift;    // cells per bucket along an axis: 2^shift
  int n_buckets;
};

static BucketGeom bucket_geom(const spl_desc* d) {
  const int n = std::max(d->grid[0], std::max(d->grid[1], d->grid[2]));
  int b = 1;
  while ((1 << b) < n) ++b;
  BucketGeom bg;
  bg.shift = b > 6 ? b - 6 : 0;
  bg.bits = b - bg.shift;
  bg.n_buckets = (1 << (3 * bg.bits)) + 1;
  return bg;
}

__global__ __launch_bounds__(256) void k_fill_zero_i32(int32_t* x, int32_t n) {  // also used by batch.hip
  for (int i = (int)(blockIdx.x * blockDim.x + threadIdx.x); i < n; i += (int)(gridDim.x * blockDim.x)) x[i] = 0;
}

__global__ __launch_bounds__(256) void k_bucket_count(Geom g, const double* pos, int32_t n_pts, int32_t shift,
                                                      int32_t sentinel, int32_t* bucket, int32_t* counts) {
  const int p = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (p >= n_pts) return;
  int i0[3];
  double t[3];
  const bool ok = reduce_point(g, pos[3 * (int64_t)p], pos[3 * (int64_t)p + 1], pos[3 * (int64_t)p + 2], i0, t);
  const int32_t b = ok ? (int32_t)((spread3((uint32_t)(i0[0] >> shift)) << 2) |
                                   (spread3((uint32_t)(i0[1] >> shift)) << 1) | spread3((uint32_t)(i0[2] >> shift)))
                       : sentinel;
  bucket[p] = b;
  atomicAdd(&counts[b], 1);
}

// offsets holds each bucket's first slot on entry and is used as its cursor.
__global__ __launch_bounds__(256) void k_bucket_scatter(int32_t n_pts, const int32_t* bucket, int32_t* offsets,
                                                        int32_t* perm) {
  const int p = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (p >= n_pts) return;
  perm[atomicAdd(&offsets[bucket[p]], 1)] = p;
}

struct PermLayout {
  size_t bucket, counts, offsets, perm, temp, temp_bytes, total;
  BucketGeom bg;
};

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

static int perm_layout(const spl_desc* d, int64_t n_pts, PermLayout* L) {
  L->bg = bucket_geom(d);
  size_t t = 0;
  int rc = hip_fail(hipcub::DeviceScan::ExclusiveSum(nullptr, t, (const int32_t*)nullptr, (int32_t*)nullptr,
                                                     L->bg.n_buckets, (hipStream_t)0),
                    "scan size query");
  if (rc) return rc;
  const size_t n = (size_t)n_pts, nb = (size_t)L->bg.n_buckets;
  size_t off = 0;
  L->bucket = off; off = align256(off + 4 * n);
  L->counts = off; off = align256(off + 4 * nb);
  L->offsets = off; off = align256(off + 4 * nb);
  L->perm = off; off = align256(off + 4 * n);
  L->temp = off; off = align256(off + t);
  L->temp_bytes = t;
  L->total = off;
  return SPL_OK;
}

int sorted_eval_work_bytes(const spl_desc* d, int64_t n_pts, int64_t* bytes) {
  PermLayout L;
  const int rc = perm_layout(d, n_pts, &L);
  if (rc) return rc;
  *bytes = (int64_t)L.total;
  return SPL_OK;
}

int launch_eval_sorted(const spl_desc* d, const void* table, int64_t n_pts, const double* pos, void* v, void* grad,
                       void* lap, int values_only, const int32_t tile[2], void* work, int64_t work_bytes,
                       hipStream_t stream) {
  if (n_pts == 0) return SPL_OK;
  PermLayout L;
  int rc = perm_layout(d, n_pts, &L);
  if (rc) return rc;
  if (work_bytes < (int64_t)L.total)
    return fail(SPL_EINVAL, "workspace of %lld bytes is smaller than the %lld needed", (long long)work_bytes,
                (long long)L.total);
  EvalKernel k = tile_valid_for(d, tile) ? eval_kernel_for(d, values_only, tile, 1) : nullptr;
  if (!k) return fail(SPL_EINVAL, "invalid tile shape (%d, %d)", tile[0], tile[1]);
  char* w = static_cast<char*>(work);
  int32_t* bucket = reinterpret_cast<int32_t*>(w + L.bucket);
  int32_t* counts = reinterpret_cast<int32_t*>(w + L.counts);
  int32_t* offsets = reinterpret_cast<int32_t*>(w + L.offsets);
  int32_t* perm = reinterpret_cast<int32_t*>(w + L.perm);
  const int nb = L.bg.n_buckets;
  const unsigned pblocks = (unsigned)((n_pts + 255) / 256);
  hipLaunchKernelGGL(k_fill_zero_i32, dim3((unsigned)std::min(1024, (nb + 255) / 256)), dim3(256), 0, stream, counts,
                     nb);
  if ((rc = hip_fail(hipGetLastError(), "bucket clear launch"))) return rc;
  const Geom geo = make_geom(d);
  hipLaunchKernelGGL(k_bucket_count, dim3(pblocks), dim3(256), 0, stream, geo, pos, (int32_t)n_pts,
                     (int32_t)L.bg.shift, (int32_t)(nb - 1), bucket, counts);
  if ((rc = hip_fail(hipGetLastError(), "bucket count launch"))) return rc;
  size_t temp_bytes = L.temp_bytes;
  if ((rc = hip_fail(hipcub::DeviceScan::ExclusiveSum(w + L.temp, temp_bytes, counts, offsets, nb, stream),
                     "bucket scan")))
    return rc;
  hipLaunchKernelGGL(k_bucket_scatter, dim3(pblocks), dim3(256), 0, stream, (int32_t)n_pts, bucket, offsets, perm);
  if ((rc = hip_fail(hipGetLastError(), "bucket scatter launch"))) return rc;
  EvalArgs a;
  fill_eval_args(d, table, n_pts, pos, v, grad, lap, values_only, tile[1], &a);
  const int64_t gpb = 256 / tile[0];
  const int64_t n_tiles = (n_pts + gpb - 1) / gpb;
  a.perm = perm;
  a.per_xcd = (int32_t)((n_tiles + 7) / 8);
  hipLaunchKernelGGL(k, dim3((unsigned)(8 * a.per_xcd)), dim3(256), 0, stream, a);
  return hip_fail(hipGetLastError(), "sorted evaluation launch");
}

// ---------------------------------------------------------------- variant that allocates nothing
// The workspace of the sorted evaluation (per-point buckets and permutation, bucket counts and
// offsets, the scan's scratch) in a fixed device array instead of a caller buffer, for callers that
// cannot allocate.  Each device holds its own copy of the array at its own address, taken once per
// device with the device current; host code uses only that address.  Every call on a device shares
// its copy, so calls that overlap on one device race.
constexpr int64_t NOALLOC_SCRATCH_BYTES = int64_t(16) << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[NOALLOC_MAX_DEVICES];

static int scratch_for_current_device(void** out) {
  int dev = -1;
  int rc = hip_fail(hipGetDevice(&dev), "hipGetDevice");
  if (rc) return rc;
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
    return fail(SPL_EUNSUPPORTED, "device %d is beyond the %d the scratch table covers", dev, NOALLOC_MAX_DEVICES);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if ((rc = hip_fail(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)"))) return rc;
    if (!p) return fail(SPL_EHIP, "hipGetSymbolAddress(scratch) returned a null address");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return SPL_OK;
}

}  // namespace pws

using namespace pws;

extern "C" int spline_eval_vgl_sorted_noalloc(const spl_desc* d, const void* table, int64_t n_pts, const double* pos,
                                              void* v, void* grad, void* lap, const int32_t* tile, void* stream) {
  clear_error();
  int rc = check_eval_args(d, table, n_pts, pos);
  if (rc) return rc;
  if (n_pts == 0) return SPL_OK;
  if ((rc = check_vgl_outputs(d, v, grad, lap))) return rc;
  int32_t t[2];
  if (tile) {
    t[0] = tile[0];
    t[1] = tile[1];
  } else {
    tile_for(d, t);
  }
  if (!tile_valid_for(d, t)) return fail(SPL_EINVAL, "invalid tile");
  PermLayout L;
  if ((rc = perm_layout(d, n_pts, &L))) return rc;
  if ((int64_t)L.total > NOALLOC_SCRATCH_BYTES)
    return fail(SPL_EINVAL, "%lld points need %lld bytes of workspace; the static scratch holds %lld bytes "
                "(about %lld points): use spline_eval_vgl_sorted with a caller workspace",
                (long long)n_pts, (long long)L.total, (long long)NOALLOC_SCRATCH_BYTES,
                (long long)((NOALLOC_SCRATCH_BYTES - ((int64_t)L.total - 8 * n_pts)) / 8));
  void* w = nullptr;
  if ((rc = scratch_for_current_device(&w))) return rc;
  return launch_eval_sorted(d, table, n_pts, pos, v, grad, lap, 0, t, w, NOALLOC_SCRATCH_BYTES,
                            static_cast<hipStream_t>(stream));
}

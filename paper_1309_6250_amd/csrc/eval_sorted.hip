// spline_eval_vgl_sorted: locality-ordered forward evaluation.
//
// Points arrive in any order (walkers x electrons, spread over the whole cell), so consecutive
// points rarely share table rows and every block is gathered from memory.  On average a row of the
// table belongs to the blocks of several points (64 P / N1 N2 N3 of them), so evaluating the points
// in the order of a space-filling curve over the grid cells lets the points that one workgroup,
// and one XCD, handle in sequence find most rows of their blocks already in L2 or the Infinity
// Cache.  Steps: a Morton key of each point's cell (three grid indices interleaved), a stable radix
// sort of (key, point index) over only the key bits the grid needs (3 x ceil(log2 max N) + 1: a
// 48^3 grid sorts 19-bit keys), then the forward kernel of the descriptor's representation through
// the permutation, with each XCD on a contiguous stretch of it.  Each point's outputs go to its own
// row, in the caller's order, with the arithmetic of the unsorted launch: bitwise the same results.
#include <hipcub/hipcub.hpp>

#include "internal.hpp"

namespace pws {

EvalKernel eval_kernel_for(const spl_desc* d, int values_only, const int32_t tile[2]);

// Spread the low 10 bits of x to every third bit.
__device__ __forceinline__ uint32_t spread3(uint32_t x) {
  x &= 0x3ffu;
  x = (x | (x << 16)) & 0x030000ffu;
  x = (x | (x << 8)) & 0x0300f00fu;
  x = (x | (x << 4)) & 0x030c30c3u;
  x = (x | (x << 2)) & 0x09249249u;
  return x;
}

// Key of a point: the Morton index of its cell (i0 interleaved, `bits` <= 10 bits per axis);
// points with non-finite coordinates get 2^(3 bits) and sort last.
__global__ __launch_bounds__(256) void k_morton_keys(Geom g, const double* pos, int32_t n_pts, int32_t bits,
                                                     uint32_t* keys, int32_t* vals) {
  const int p = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (p >= n_pts) return;
  int i0[3];
  double t[3];
  const bool ok = reduce_point(g, pos[3 * (int64_t)p], pos[3 * (int64_t)p + 1], pos[3 * (int64_t)p + 2], i0, t);
  keys[p] = ok ? (spread3((uint32_t)i0[0]) << 2) | (spread3((uint32_t)i0[1]) << 1) | spread3((uint32_t)i0[2])
               : (1u << (3 * bits));
  vals[p] = p;
}

struct PermLayout {
  size_t keys_in, keys_out, vals_in, vals_out, temp, temp_bytes, total;
};

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Bits per axis of the Morton key: enough for the largest grid index.
static int key_bits(const spl_desc* d) {
  const int n = std::max(d->grid[0], std::max(d->grid[1], d->grid[2]));
  int b = 1;
  while ((1 << b) < n) ++b;
  return b;
}

static int perm_layout(const spl_desc* d, int64_t n_pts, PermLayout* L) {
  size_t t = 0;
  const int end_bit = 3 * key_bits(d) + 1;
  int rc = hip_fail(hipcub::DeviceRadixSort::SortPairs(nullptr, t, (const uint32_t*)nullptr, (uint32_t*)nullptr,
                                                       (const int32_t*)nullptr, (int32_t*)nullptr, (int)n_pts, 0,
                                                       end_bit, (hipStream_t)0),
                    "radix sort size query");
  if (rc) return rc;
  const size_t n = (size_t)n_pts;
  size_t off = 0;
  L->keys_in = off; off = align256(off + 4 * n);
  L->keys_out = off; off = align256(off + 4 * n);
  L->vals_in = off; off = align256(off + 4 * n);
  L->vals_out = off; off = align256(off + 4 * n);
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
  EvalKernel k = tile_valid_for(d, tile) ? eval_kernel_for(d, values_only, tile) : nullptr;
  if (!k) return fail(SPL_EINVAL, "invalid tile shape (%d, %d)", tile[0], tile[1]);
  char* w = static_cast<char*>(work);
  uint32_t* keys_in = reinterpret_cast<uint32_t*>(w + L.keys_in);
  uint32_t* keys_out = reinterpret_cast<uint32_t*>(w + L.keys_out);
  int32_t* vals_in = reinterpret_cast<int32_t*>(w + L.vals_in);
  int32_t* vals_out = reinterpret_cast<int32_t*>(w + L.vals_out);
  const Geom geo = make_geom(d);
  const int bits = key_bits(d);
  hipLaunchKernelGGL(k_morton_keys, dim3((unsigned)((n_pts + 255) / 256)), dim3(256), 0, stream, geo, pos,
                     (int32_t)n_pts, (int32_t)bits, keys_in, vals_in);
  if ((rc = hip_fail(hipGetLastError(), "cell key launch"))) return rc;
  size_t temp_bytes = L.temp_bytes;
  if ((rc = hip_fail(hipcub::DeviceRadixSort::SortPairs(w + L.temp, temp_bytes, keys_in, keys_out, vals_in, vals_out,
                                                        (int)n_pts, 0, 3 * bits + 1, stream),
                     "radix sort")))
    return rc;
  EvalArgs a;
  fill_eval_args(d, table, n_pts, pos, v, grad, lap, values_only, tile[1], &a);
  const int64_t gpb = 256 / tile[0];
  const int64_t n_tiles = (n_pts + gpb - 1) / gpb;
  a.perm = vals_out;
  a.per_xcd = (int32_t)((n_tiles + 7) / 8);
  hipLaunchKernelGGL(k, dim3((unsigned)(8 * a.per_xcd)), dim3(256), 0, stream, a);
  return hip_fail(hipGetLastError(), "sorted evaluation launch");
}

}  // namespace pws

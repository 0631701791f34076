// Deterministic coefficient gradient of spline_eval_vgl_backward (flag SPL_DETERMINISTIC).
//
// The gradient of a coefficient is a sum over every point whose 4x4x4 block contains it.
// Float atomics make the order of that sum, and so its rounding, depend on scheduling.  Here:
//
//  1. every point gets the key (colour class, cell) of the grid cell it falls in; points with
//     non-finite coordinates get a key past all classes;
//  2. a stable radix sort orders points by key (then by index), and a run-length encoding
//     lists the occupied cells with the range of their points;
//  3. for each colour class in turn, one lane group per (cell, orbital chunk) accumulates the
//     contributions of all of the cell's points to its 64 rows in registers, in point order,
//     then adds them to the gradient table with ordinary loads and stores.
//
// Colour classes: along an axis of N cells, cell i has colour i mod 4 when i < 4 floor(N/4), and
// a colour of its own (4, 5, 6) for the last N mod 4 cells.  Two cells of one class are at least
// 4 apart along every axis, also across the periodic wrap, so their blocks (rows i-1 .. i+2) are
// disjoint: within a class no two lane groups touch the same row, and classes run one after the
// other.  The result is bitwise reproducible, and each row is written once per occupied cell
// rather than once per point.
#include <hipcub/hipcub.hpp>

#include "common.hpp"

namespace pws {

__host__ __device__ inline int axis_colour(int i, int n) {
  const int full = n & ~3;
  return i < full ? (i & 3) : 4 + (i - full);
}
__host__ __device__ inline int axis_colours(int n) { return 4 + (n & 3); }

struct SortLayout {
  size_t keys_in, keys_out, vals_in, vals_out, uniq, counts, offsets, num_runs, class_start, temp;
  size_t temp_bytes, total;
  int n_classes;
  int64_t n_cells;
  int end_bit;
};

static size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

static int sort_layout(const spl_desc* d, int64_t n_pts, SortLayout* L) {
  L->n_cells = (int64_t)d->grid[0] * d->grid[1] * d->grid[2];
  L->n_classes = axis_colours(d->grid[0]) * axis_colours(d->grid[1]) * axis_colours(d->grid[2]);
  const uint64_t max_key = (uint64_t)(L->n_classes + 1) * (uint64_t)L->n_cells;
  int bits = 1;
  while (bits < 63 && ((uint64_t)1 << bits) <= max_key) ++bits;
  L->end_bit = bits;
  const size_t n = (size_t)n_pts;
  size_t t1 = 0, t2 = 0, t3 = 0;
  int rc = hip_fail(hipcub::DeviceRadixSort::SortPairs(nullptr, t1, (const int64_t*)nullptr, (int64_t*)nullptr,
                                                       (const int32_t*)nullptr, (int32_t*)nullptr, (int)n, 0,
                                                       L->end_bit, (hipStream_t)0),
                    "radix sort size query");
  if (rc) return rc;
  rc = hip_fail(hipcub::DeviceRunLengthEncode::Encode(nullptr, t2, (const int64_t*)nullptr, (int64_t*)nullptr,
                                                      (int32_t*)nullptr, (int32_t*)nullptr, (int)n, (hipStream_t)0),
                "run-length encode size query");
  if (rc) return rc;
  rc = hip_fail(hipcub::DeviceScan::ExclusiveSum(nullptr, t3, (const int32_t*)nullptr, (int32_t*)nullptr, (int)n,
                                                 (hipStream_t)0),
                "scan size query");
  if (rc) return rc;
  L->temp_bytes = std::max(t1, std::max(t2, t3));
  size_t off = 0;
  L->keys_in = off; off = align_up(off + 8 * n);
  L->keys_out = off; off = align_up(off + 8 * n);
  L->vals_in = off; off = align_up(off + 4 * n);
  L->vals_out = off; off = align_up(off + 4 * n);
  L->uniq = off; off = align_up(off + 8 * n);
  L->counts = off; off = align_up(off + 4 * n);
  L->offsets = off; off = align_up(off + 4 * n);
  L->num_runs = off; off = align_up(off + 4);
  L->class_start = off; off = align_up(off + 4 * (size_t)(L->n_classes + 2));
  L->temp = off; off = align_up(off + L->temp_bytes);
  L->total = off;
  return SPL_OK;
}

__global__ __launch_bounds__(256) void k_cell_keys(Geom g, const double* pos, int32_t n_pts, int64_t n_cells,
                                                   int64_t sentinel, int64_t* keys, int32_t* vals) {
  const int p = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (p >= n_pts) return;
  int i0[3];
  double t[3];
  const bool ok = reduce_point(g, pos[3 * (int64_t)p], pos[3 * (int64_t)p + 1], pos[3 * (int64_t)p + 2], i0, t);
  const int64_t cell = ((int64_t)i0[0] * g.n[1] + i0[1]) * g.n[2] + i0[2];
  const int c1 = axis_colours(g.n[1]), c2 = axis_colours(g.n[2]);
  const int64_t cls = ((int64_t)axis_colour(i0[0], g.n[0]) * c1 + axis_colour(i0[1], g.n[1])) * c2 +
                      axis_colour(i0[2], g.n[2]);
  keys[p] = ok ? cls * n_cells + cell : sentinel;
  vals[p] = p;
}

// class_start[c] = first run whose key belongs to class c or later (c = 0 .. n_classes)
__global__ void k_class_starts(const int64_t* uniq, const int32_t* num_runs, int64_t n_cells, int32_t n_classes,
                               int32_t* class_start) {
  const int c = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (c > n_classes) return;
  const int64_t key = (int64_t)c * n_cells;
  int lo = 0, hi = *num_runs;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (uniq[mid] < key) lo = mid + 1;
    else hi = mid;
  }
  class_start[c] = lo;
}

struct CellArgs {
  Geom g;
  const double* pos;
  const void* gv;
  const void* ggrad;
  const void* glap;
  void* gtable;        // base of the table this pass writes (orbital or Laplacian table)
  const int64_t* uniq;
  const int32_t* counts;
  const int32_t* offsets;
  const int32_t* perm;
  const int32_t* class_start;
  int64_t n_cells;
  int32_t cls;
  int32_t n_orb;
  int32_t n_chunks;
  int32_t pad_;
};

template <typename A>
__device__ __forceinline__ A pick4c(int l, A a0, A a1, A a2, A a3) {
  return l == 0 ? a0 : (l == 1 ? a1 : (l == 2 ? a2 : a3));
}

// SEPLAP: the Laplacian's gradient goes to the separate table (orbital pass ignores gL);
// LAPTAB: this pass accumulates the separate Laplacian table (value weights times gL).
template <typename TS, bool SEPLAP, bool LAPTAB, int G, int OPL>
__global__ __launch_bounds__(256) void k_bwd_cells(CellArgs a) {
  using A = typename Acc<TS>::type;
  using GO = typename Out<TS>::type;
  constexpr int GPB = 256 / G;
  const int grp = threadIdx.x / G;
  const int lane = threadIdx.x % G;
  const int r0 = a.class_start[a.cls];
  const int r1 = a.class_start[a.cls + 1];
  const int64_t n_work = (int64_t)(r1 - r0) * a.n_chunks;
  const GO* gvp = static_cast<const GO*>(a.gv);
  const GO* ggp = static_cast<const GO*>(a.ggrad);
  const GO* glp = static_cast<const GO*>(a.glap);
  GO* gtab = static_cast<GO*>(a.gtable);
  A jm[9], mt[6];
#pragma unroll
  for (int i = 0; i < 9; ++i) jm[i] = (A)a.g.jac[i];
#pragma unroll
  for (int i = 0; i < 6; ++i) mt[i] = (A)a.g.metric[i];

  for (int64_t w = (int64_t)blockIdx.x * GPB + grp; w < n_work; w += (int64_t)gridDim.x * GPB) {
    const int r = r0 + (int)(w / a.n_chunks);
    const int cb = (int)(w % a.n_chunks) * G * OPL;
    const int64_t cell = a.uniq[r] - (int64_t)a.cls * a.n_cells;
    const int iz0 = (int)(cell % a.g.n[2]);
    const int iy0 = (int)((cell / a.g.n[2]) % a.g.n[1]);
    const int ix0 = (int)(cell / ((int64_t)a.g.n[2] * a.g.n[1]));
    int ix[4], iy[4], iz[4];
    wrap4(ix0, a.g.n[0], ix);
    wrap4(iy0, a.g.n[1], iy);
    wrap4(iz0, a.g.n[2], iz);
    int oj[OPL];
    bool inj[OPL];
#pragma unroll
    for (int j = 0; j < OPL; ++j) {
      oj[j] = cb + lane + j * G;
      inj[j] = oj[j] < a.n_orb;
    }
    A acc[64][OPL];
#pragma unroll
    for (int q = 0; q < 64; ++q)
#pragma unroll
      for (int j = 0; j < OPL; ++j) acc[q][j] = A(0);

    const int start = a.offsets[r];
    const int cnt = a.counts[r];
    for (int i = 0; i < cnt; ++i) {
      const int p = a.perm[start + i];
      int i0[3];
      double t[3];
      reduce_point(a.g, a.pos[3 * (int64_t)p], a.pos[3 * (int64_t)p + 1], a.pos[3 * (int64_t)p + 2], i0, t);
      A wx[4], wy[4], wz[4], dwx[4], dwy[4], dwz[4], d2wx[4], d2wy[4], d2wz[4];
      bspline_weights<A>((A)t[0], wx, dwx, d2wx);
      bspline_weights<A>((A)t[1], wy, dwy, d2wy);
      bspline_weights<A>((A)t[2], wz, dwz, d2wz);
#pragma unroll
      for (int j = 0; j < OPL; ++j) {
        const bool in = inj[j];
        const int64_t po = (int64_t)p * a.n_orb + oj[j];
        const int64_t pg = (int64_t)p * 3 * a.n_orb + oj[j];
        const A gL = (in && glp) ? (A)glp[po] : A(0);
        if constexpr (LAPTAB) {
#pragma unroll
          for (int l = 0; l < 4; ++l)
#pragma unroll
            for (int m = 0; m < 4; ++m) {
              const A xy = gL * (wx[l] * wy[m]);
#pragma unroll
              for (int n = 0; n < 4; ++n) acc[(l * 4 + m) * 4 + n][j] = fmaa(xy, wz[n], acc[(l * 4 + m) * 4 + n][j]);
            }
        } else {
          const A gV = (in && gvp) ? (A)gvp[po] : A(0);
          const A g0 = (in && ggp) ? (A)ggp[pg] : A(0);
          const A g1 = (in && ggp) ? (A)ggp[pg + a.n_orb] : A(0);
          const A g2 = (in && ggp) ? (A)ggp[pg + 2 * a.n_orb] : A(0);
          A gt[3];
#pragma unroll
          for (int k = 0; k < 3; ++k) gt[k] = fmaa(jm[3 * k + 2], g2, fmaa(jm[3 * k + 1], g1, jm[3 * k] * g0));
          const A cl = SEPLAP ? A(0) : gL;
#pragma unroll
          for (int l = 0; l < 4; ++l) {
            const A e0 = fmaa(mt[0] * cl, d2wx[l], fmaa(gt[0], dwx[l], gV * wx[l]));
            const A e1 = fmaa(A(2) * mt[3] * cl, dwx[l], gt[1] * wx[l]);
            const A e2 = fmaa(A(2) * mt[4] * cl, dwx[l], gt[2] * wx[l]);
            const A e3 = (mt[1] * cl) * wx[l];
            const A e4 = (mt[2] * cl) * wx[l];
            const A e5 = (A(2) * mt[5] * cl) * wx[l];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
              const A f0 = fmaa(e3, d2wy[m], fmaa(e1, dwy[m], e0 * wy[m]));
              const A f1 = fmaa(e5, dwy[m], e2 * wy[m]);
              const A f2 = e4 * wy[m];
#pragma unroll
              for (int n = 0; n < 4; ++n)
                acc[(l * 4 + m) * 4 + n][j] += fmaa(f2, d2wz[n], fmaa(f1, dwz[n], f0 * wz[n]));
            }
          }
        }
      }
    }
    // this cell's block: no other lane group of the class touches these rows
#pragma unroll
    for (int l = 0; l < 4; ++l)
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        GO* rp = gtab + (int64_t)ix[l] * a.g.s0 + (int64_t)iy[m] * a.g.s1;
#pragma unroll
        for (int n = 0; n < 4; ++n)
#pragma unroll
          for (int j = 0; j < OPL; ++j)
            if (inj[j]) {
              GO* q = rp + (int64_t)iz[n] * a.g.o_pad + oj[j];
              *q = *q + (GO)acc[(l * 4 + m) * 4 + n][j];
            }
      }
  }
}

typedef void (*CellKernel)(CellArgs);

template <typename TS, bool SEPLAP, bool LAPTAB>
static CellKernel pick_cells(int g) {
  switch (g) {
    case 4: return k_bwd_cells<TS, SEPLAP, LAPTAB, 4, 1>;
    case 16: return k_bwd_cells<TS, SEPLAP, LAPTAB, 16, 1>;
    default: return k_bwd_cells<TS, SEPLAP, LAPTAB, 64, 1>;
  }
}

template <typename TS>
static CellKernel pick_cells_t(bool seplap, bool laptab, int g) {
  if (laptab) return pick_cells<TS, true, true>(g);
  return seplap ? pick_cells<TS, true, false>(g) : pick_cells<TS, false, false>(g);
}

int sorted_work_bytes(const spl_desc* d, int64_t n_pts, int64_t* bytes) {
  SortLayout L;
  int rc = sort_layout(d, n_pts, &L);
  if (rc) return rc;
  *bytes = (int64_t)L.total;
  return SPL_OK;
}

// Deterministic coefficient gradient (accumulated into gtable).  work: sorted_work_bytes bytes.
int launch_backward_sorted(const spl_desc* d, int64_t n_pts, const double* pos, const void* gv, const void* ggrad,
                           const void* glap, void* gtable, void* work, int64_t work_bytes, hipStream_t stream) {
  if (n_pts == 0 || !gtable) return SPL_OK;
  SortLayout L;
  int rc = sort_layout(d, n_pts, &L);
  if (rc) return rc;
  if (!work || work_bytes < (int64_t)L.total)
    return fail(SPL_EINVAL, "deterministic backward needs a workspace of %lld bytes", (long long)L.total);
  char* W = static_cast<char*>(work);
  int64_t* keys_in = reinterpret_cast<int64_t*>(W + L.keys_in);
  int64_t* keys_out = reinterpret_cast<int64_t*>(W + L.keys_out);
  int32_t* vals_in = reinterpret_cast<int32_t*>(W + L.vals_in);
  int32_t* vals_out = reinterpret_cast<int32_t*>(W + L.vals_out);
  int64_t* uniq = reinterpret_cast<int64_t*>(W + L.uniq);
  int32_t* counts = reinterpret_cast<int32_t*>(W + L.counts);
  int32_t* offsets = reinterpret_cast<int32_t*>(W + L.offsets);
  int32_t* num_runs = reinterpret_cast<int32_t*>(W + L.num_runs);
  int32_t* class_start = reinterpret_cast<int32_t*>(W + L.class_start);
  void* temp = W + L.temp;
  const Geom g = make_geom(d);
  const int n = (int)n_pts;
  hipLaunchKernelGGL(k_cell_keys, dim3((n + 255) / 256), dim3(256), 0, stream, g, pos, (int32_t)n, L.n_cells,
                     (int64_t)L.n_classes * L.n_cells, keys_in, vals_in);
  if ((rc = hip_fail(hipGetLastError(), "cell key launch"))) return rc;
  size_t tb = L.temp_bytes;
  if ((rc = hip_fail(hipcub::DeviceRadixSort::SortPairs(temp, tb, keys_in, keys_out, vals_in, vals_out, n, 0,
                                                        L.end_bit, stream), "radix sort")))
    return rc;
  tb = L.temp_bytes;
  if ((rc = hip_fail(hipcub::DeviceRunLengthEncode::Encode(temp, tb, keys_out, uniq, counts, num_runs, n, stream),
                     "run-length encode")))
    return rc;
  tb = L.temp_bytes;
  if ((rc = hip_fail(hipcub::DeviceScan::ExclusiveSum(temp, tb, counts, offsets, n, stream), "scan"))) return rc;
  hipLaunchKernelGGL(k_class_starts, dim3((L.n_classes + 1 + 255) / 256), dim3(256), 0, stream, uniq, num_runs,
                     L.n_cells, (int32_t)L.n_classes, class_start);
  if ((rc = hip_fail(hipGetLastError(), "class start launch"))) return rc;

  const int gl = d->n_orb <= 4 ? 4 : (d->n_orb <= 16 ? 16 : 64);
  CellArgs a;
  a.g = g;
  a.pos = pos;
  a.gv = gv;
  a.ggrad = ggrad;
  a.glap = glap;
  a.uniq = uniq;
  a.counts = counts;
  a.offsets = offsets;
  a.perm = vals_out;
  a.class_start = class_start;
  a.n_cells = L.n_cells;
  a.n_orb = d->n_orb;
  a.n_chunks = (d->n_orb + gl - 1) / gl;
  a.pad_ = 0;
  const int passes = d->has_lap ? 2 : 1;
  const size_t gsz = d->dtype == SPL_F64 ? 8 : 4;
  for (int pass = 0; pass < passes; ++pass) {
    const bool laptab = pass == 1;
    a.gtable = static_cast<char*>(gtable) + (laptab ? d->table_elems * gsz : 0);
    CellKernel k;
    if (d->dtype == SPL_F64) k = pick_cells_t<double>(d->has_lap, laptab, gl);
    else if (d->dtype == SPL_F32) k = pick_cells_t<float>(d->has_lap, laptab, gl);
    else k = pick_cells_t<uint16_t>(d->has_lap, laptab, gl);
    for (int c = 0; c < L.n_classes; ++c) {
      a.cls = c;
      hipLaunchKernelGGL(k, dim3(512), dim3(256), 0, stream, a);
      if ((rc = hip_fail(hipGetLastError(), "cell gradient launch"))) return rc;
    }
  }
  return SPL_OK;
}

}  // namespace pws

// Work on the points grouped by grid cell: the deterministic coefficient gradient of
// spline_eval_vgl_backward (flag SPL_DETERMINISTIC) and the cell-wise forward evaluation
// spline_eval_vgl_cells.  Both start from the same sort:
//
//  1. every point gets the index of the grid cell it falls in as its key; points with non-finite
//     coordinates get a key past all cells;
//  2. a stable radix sort orders points by key (then by index), a run-length encoding lists the
//     occupied cells with the range of their points, and each sorted point gets a record of its
//     reduced coordinates and index.
//
// Summed over the points of one cell, both directions are dense products between the cell's 64
// block rows and its points (row weights from the 1-D B-spline weights), done on the matrix cores.
//
// Adjoint.  The gradient of a coefficient is a sum over every point whose 4x4x4 block contains it;
// float atomics would make its order, and so its rounding, depend on scheduling.  Here every sum
// is formed in a fixed order, either
//  - with 2.5 or more points per cell, cell by cell: each cell's block in point order, summed per
//    brick of 2 x 2 x 2 cells into the workspace, followed by a gather in which every table row
//    sums the brick regions that contain it in a fixed order; or
//  - with fewer, tile by tile: each tile of 4 x 4 x 4 rows sums the points of the cells whose
//    blocks reach it, in cell and point order, and adds the sum to its rows once.
// Either way the result is reproducible bit for bit.
//
// Forward.  A wave loads a cell's block once and multiplies it with the row weights of the
// cell's points, so each block row is read once per cell instead of once per point.  For the
// least-squares fit (spline_fit_terms_cells) the same kernel compares its outputs with targets as it
// writes them: it stores the misfit's upstream gradients instead of the outputs and adds the squared
// residuals to one FP64 partial sum per work item, summed afterwards in a fixed order.
#include <hipcub/hipcub.hpp>
#include <rocprim/device/device_radix_sort.hpp>

#include <algorithm>
#include <cstring>

#include "cells.hpp"
#include "common.hpp"

namespace pws {

struct SortLayout {
  size_t keys_in, keys_out, vals_in, vals_out, uniq, counts, offsets, num_runs, finite_runs, pts, cell_range, blocks,
      partials, temp;
  size_t temp_bytes, total;
  int dense;           // 1: brick regions in the workspace and a per-row gather instead of row tiles
  int64_t n_cells;
  int end_bit;
};

static size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// The stable sort of the cell keys (point index as value).  rocPRIM's radix sort uses a block sort
// followed by merge passes up to 2^20 items; at the fit's 10^6 points that path took about 190 us
// (ten merge passes) and onesweep about 100 us less, while at 65 536 points the merge path is the
// faster by about 40 us.  So merge sort up to 2^18 items, onesweep above.  Both are stable: the
// sorted order, and every sum formed in it, is the same either way.
using CellSortConfig = rocprim::radix_sort_config<rocprim::default_config, rocprim::default_config,
                                                  rocprim::default_config, (size_t)1 << 18>;
static hipError_t sort_cell_keys(void* temp, size_t& bytes, const int64_t* keys_in, int64_t* keys_out,
                                 const int32_t* vals_in, int32_t* vals_out, int n, int end_bit, hipStream_t stream) {
  return rocprim::radix_sort_pairs<CellSortConfig>(temp, bytes, keys_in, keys_out, vals_in, vals_out, n, 0,
                                                   (unsigned)end_bit, stream);
}

// the fit terms' loss: workgroups of the first summing step, and threads of both steps
constexpr int FIT_SUM_BLOCKS = 256;
constexpr int FIT_SUM_THREADS = 256;

static int sort_layout(const spl_desc* d, int64_t n_pts, SortLayout* L, bool adjoint_blocks = true,
                       bool fit_partials = false) {
  L->n_cells = (int64_t)d->grid[0] * d->grid[1] * d->grid[2];
  const uint64_t max_key = (uint64_t)L->n_cells;     // the non-finite points' key
  int bits = 1;
  while (bits < 63 && ((uint64_t)1 << bits) <= max_key) ++bits;
  L->end_bit = bits;
  const size_t n = (size_t)n_pts;
  size_t t1 = 0, t2 = 0, t3 = 0;
  int rc = hip_fail(sort_cell_keys(nullptr, t1, nullptr, nullptr, nullptr, nullptr, (int)n, L->end_bit, nullptr),
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
  L->finite_runs = off; off = align_up(off + 4);
  L->pts = off; off = align_up(off + (d->dtype == SPL_F64 ? 32 : 16) * n);
  // dense points (at least 4 per cell on average): the 5 x 5 x 5-row region of every brick of 2 x 2 x 2
  // cells gets its own place, and every cell its sorted point range
  const size_t gsz = d->dtype == SPL_F64 ? 8 : 4;
  const size_t n_bricks = (size_t)((d->grid[0] + 1) / 2) * ((d->grid[1] + 1) / 2) * ((d->grid[2] + 1) / 2);
  const size_t block_bytes = n_bricks * 125 * (size_t)d->o_pad * gsz;
  // (the crossover of the two forms measured on the Si-like cell: 1.7 to 2.7 points per cell, by term set
  // and precision)
  L->dense = adjoint_blocks && 2 * n_pts >= 5 * L->n_cells && block_bytes <= ((size_t)4 << 30);
  // every cell's sorted point range: the adjoint's brick and row-tile forms both look cells up
  L->cell_range = off; off = align_up(off + (adjoint_blocks ? 12 * (size_t)L->n_cells : 0));
  L->blocks = off; off = align_up(off + (L->dense ? block_bytes : 0));
  // the fit terms: one FP64 partial sum per work item, at most min(n, cells) runs times the 16-orbital
  // tiles, then one per workgroup of the first summing step (FIT_SUM_BLOCKS)
  L->partials = off;
  if (!adjoint_blocks || fit_partials)
    off = align_up(off + 8 * ((size_t)std::min<int64_t>(n_pts, L->n_cells) * (size_t)((d->n_orb + 15) / 16) + FIT_SUM_BLOCKS));
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
  keys[p] = ok ? cell : sentinel;
  vals[p] = p;
}

// finite_runs = the runs of finite points (occupied cells): the first run whose key is n_cells or more
__global__ void k_finite_runs(const int64_t* uniq, const int32_t* num_runs, int64_t n_cells, int32_t* finite_runs) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  int lo = 0, hi = *num_runs;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (uniq[mid] < n_cells) lo = mid + 1;
    else hi = mid;
  }
  *finite_runs = lo;
}

// A point in sorted order: its reduced coordinates within its cell and its index.
template <typename A>
struct SortedPoint {
  A t[3];
  int32_t p;
};
static_assert(sizeof(SortedPoint<float>) == 16 && sizeof(SortedPoint<double>) == 32, "sorted point record size");

template <typename A>
__global__ __launch_bounds__(256) void k_sorted_points(Geom g, const double* pos, const int32_t* perm, int32_t n,
                                                       SortedPoint<A>* out) {
  const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i >= n) return;
  const int p = perm[i];
  int i0[3];
  double t[3];
  reduce_point(g, pos[3 * (int64_t)p], pos[3 * (int64_t)p + 1], pos[3 * (int64_t)p + 2], i0, t);
  SortedPoint<A> sp;
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) sp.t[ax] = (A)t[ax];
  sp.p = p;
  out[i] = sp;
}

// Terms of the upstream gradient: the value, the three Cartesian gradient components and the
// Laplacian.  Each has its own weight on the 64 rows of a block (the transpose of its row of
// the forward contraction).
enum { TERM_VAL = 0, TERM_GX = 1, TERM_GY = 2, TERM_GZ = 3, TERM_LAP = 4 };

struct CellArgs {
  Geom g;
  const double* pos;
  const void* src[5];      // upstream gradient of each term, point-major, in the gradient type
  int64_t src_stride[5];   // elements from one point to the next (n_orb, or 3 n_orb for the gradient)
  int32_t kind[5];         // TERM_* of each term
  int32_t n_terms;
  void* gtable;            // base of the table this pass writes (orbital or Laplacian table)
  const void* pts;         // SortedPoint records in sorted order
  int64_t n_cells;
  int32_t n_orb;
  int32_t n_groups;        // orbital groups of 16 OT per cell
  int32_t n_pts;           // every index read from the sort is checked against this and n_cells
  int32_t o_pad;
  void* blocks;              // dense: [n_bricks][125][o_pad] gradient regions of the bricks of 2 x 2 x 2 cells
  const int32_t* cell_range; // [n_cells][3] first sorted point, count (0 if empty) and run of each cell
  int32_t src_bytes[5];      // bytes of each term's upstream array from src[c] to its last value, or -1
                             // when one reaches 2 GiB (then the brick and tile kernels use 64-bit addresses)
};

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// 16x16x4 matrix-core step D = A B + C in the gradient's precision.  Operand layout of one
// wave: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16].  Element r of lane l's
// accumulator is D[row(l / 16, r)][l % 16], with row = 4 (l / 16) + r for FP32 and
// (l / 16) + 4 r for FP64.
template <typename A> struct Mfma;
template <> struct Mfma<float> {
  using acc = f32x4;
  __device__ __forceinline__ static int row(int grp, int r) { return 4 * grp + r; }
  __device__ __forceinline__ static acc step(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <> struct Mfma<double> {
  using acc = f64x4;
  __device__ __forceinline__ static int row(int grp, int r) { return grp + 4 * r; }
  __device__ __forceinline__ static acc step(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

// Row-weight factors of one term on a lane's (m, n) pair of block offsets: the weight of block row
// (l, m, n) is Q0 w_x[l] + Q1 w_x'[l] + Q2 w_x''[l], from the point's 1-D weights on the second and
// third axes (the transpose of the term's row of the forward contraction with the chain rule).
template <typename A>
__device__ __forceinline__ void term_factors(int kind, A wy, A dwy, A d2wy, A wz, A dwz, A d2wz, const A (&jm)[9],
                                             const A (&mt)[6], A& q0, A& q1, A& q2) {
  const A yz = wy * wz;
  q1 = A(0);
  q2 = A(0);
  if (kind == TERM_VAL) {
    q0 = yz;
  } else if (kind == TERM_LAP) {
    q2 = mt[0] * yz;
    q1 = A(2) * fmaa(mt[3] * dwy, wz, mt[4] * wy * dwz);
    q0 = fmaa(mt[1] * d2wy, wz, fmaa(mt[2] * wy, d2wz, A(2) * mt[5] * dwy * dwz));
  } else {
    const int k = kind - TERM_GX;
    q1 = jm[k] * yz;
    q0 = fmaa(jm[3 + k] * dwy, wz, jm[6 + k] * wy * dwz);
  }
}

// The adjoint's points are taken in batches: a batch's point records and 1-D weights are staged in
// LDS once and shared by the waves of a workgroup, four points per matrix-core step.
constexpr int CELL_PB = 32;         // most points per batch

// Dense points (2.5 or more per cell): the cells are taken in bricks of 2 x 2 x 2 (the last brick of
// an axis with an odd count holds one cell along it).  The blocks of a brick's cells cover a
// region of 5 x 5 x 5 table rows (rows 2 b - 1 .. 2 b + 3 along each axis, before the periodic
// wrap).  One workgroup of BRICK_WAVES waves per (brick, group of BRICK_WAVES x 16 OT orbitals)
// forms every cell's block (each wave for its own 16 OT orbitals) and adds it into its columns of
// the region, held in LDS; the region then goes to the workspace once.  A second kernel gathers,
// for every table row, the regions of the bricks that cover it.  So each table row crosses memory
// about 2^3 to 3^3 times instead of 64 times (once per cell block containing it), and the order of
// every sum stays fixed.
//
// The brick's points are taken in batches of at most CELL_PB (the cells in a fixed order, each
// cell's points in sorted order), and the memory accesses of later batches overlap the matrix-core
// work of the current one: the cells' point ranges come in one load per brick; the first 3 CELL_PB
// threads (one per point and axis) hold the sorted-point records of the next two batches in
// registers, loaded while the batch before is multiplied, and stage each batch's indices and 1-D
// weights in LDS; and (with at most two terms) every wave loads the next batch's upstream values
// before it multiplies the current one.
constexpr int BRICK_ROWS = 125;
constexpr int BRICK_WAVES = 4;

// A 4- or 8-byte load through a raw buffer resource (a byte offset past the resource's size reads 0).
template <typename A> struct BufLoad;
template <> struct BufLoad<float> {
  __device__ __forceinline__ static float load(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0));
  }
};
template <> struct BufLoad<double> {
  __device__ __forceinline__ static double load(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0));
  }
};

// The term set of the fit (value and Laplacian upstream gradients, in that order), the full set
// (value, the three gradient components and the Laplacian, in that order) and a value term alone
// (the separate Laplacian table's pass) take their row weights without a choice at run time; any
// other set reads each term's kind from CellArgs.  TSET_VLD is the fit's pair for a diagonal metric
// (orthogonal lattice vectors) and TSET_ALLD the full set for a diagonal Jacobian (orthogonal
// vectors along the Cartesian axes): the products of the zero entries, exact zeros in the general
// form, are skipped, which gives the same numbers (an exact zero may differ in sign).
enum { TSET_ANY = 0, TSET_VL = 1, TSET_ALL = 2, TSET_V = 3, TSET_VLD = 4, TSET_ALLD = 5 };

// The Laplacian's row-weight factors for a diagonal metric (M01 = M02 = M12 = 0): Q1 = 0, and Q0
// without its 2 M12 w_y' w_z' term; the general form's products of those zeros change no nonzero
// value.
template <typename A>
__device__ __forceinline__ void lap_factors_diag(A wy, A d2wy, A wz, A d2wz, const A (&mt)[6], A& q0, A& q1, A& q2) {
  q2 = mt[0] * (wy * wz);
  q1 = A(0);
  q0 = fmaa(mt[1] * d2wy, wz, (mt[2] * wy) * d2wz);
}

// Whether the kernels' diagonal forms apply: the metric's off-diagonal entries (diag), and also the
// Jacobian's (diag_jac), are zero as the kernels round them (FP64 for FP64 tables, else FP32).
struct DiagForms {
  bool diag, diag_jac;
};
static DiagForms diag_forms(const spl_desc* d) {
  auto zero = [&](double x) { return d->dtype == SPL_F64 ? x == 0.0 : (float)x == 0.0f; };
  DiagForms f;
  f.diag = zero(d->metric[3]) && zero(d->metric[4]) && zero(d->metric[5]);
  f.diag_jac = f.diag && zero(d->jac[1]) && zero(d->jac[2]) && zero(d->jac[3]) && zero(d->jac[5]) &&
               zero(d->jac[6]) && zero(d->jac[7]);
  return f;
}

// The weights of term c (kind `kind`) on a lane's four block rows l = 0..3 along the first axis,
// at its second- and third-axis offsets with 1-D weights (wy, wy', wy'') and (wz, wz', wz''):
// Q0 w_x[l] + Q1 w_x'[l] + Q2 w_x''[l].  A fixed set's value term is Q0 w_x (Q1 = Q2 = 0: with
// finite non-negative weights the two vanishing products change no bit).  With a diagonal Jacobian a
// gradient term is one product (x: Q1 = J00 w_y w_z; y: Q0 = J11 w_y' w_z; z: Q0 = J22 w_y w_z'), and
// with a diagonal metric the Laplacian has no Q1 (lap_factors_diag).
template <typename A, int TSET>
__device__ __forceinline__ void row_weights(int c, int kind, const A (&wx)[4], const A (&dwx)[4], const A (&d2wx)[4],
                                            A wy, A dwy, A d2wy, A wz, A dwz, A d2wz, const A (&jm)[9],
                                            const A (&mt)[6], A (&av)[4]) {
  if (TSET != TSET_ANY && c == 0) {
    const A q0 = wy * wz;
#pragma unroll
    for (int l = 0; l < 4; ++l) av[l] = q0 * wx[l];
  } else if (TSET == TSET_ALLD && c >= 1 && c <= 3) {
    const A q = c == 1 ? jm[0] * (wy * wz) : (c == 2 ? (jm[4] * dwy) * wz : (jm[8] * wy) * dwz);
#pragma unroll
    for (int l = 0; l < 4; ++l) av[l] = q * (c == 1 ? dwx[l] : wx[l]);
  } else if ((TSET == TSET_VLD && c == 1) || (TSET == TSET_ALLD && c == 4)) {
    A q0, q1, q2;
    lap_factors_diag<A>(wy, d2wy, wz, d2wz, mt, q0, q1, q2);
#pragma unroll
    for (int l = 0; l < 4; ++l) av[l] = fmaa(q2, d2wx[l], q0 * wx[l]);
  } else {
    A q0, q1, q2;
    term_factors<A>(kind, wy, dwy, d2wy, wz, dwz, d2wz, jm, mt, q0, q1, q2);
#pragma unroll
    for (int l = 0; l < 4; ++l) av[l] = fmaa(q2, d2wx[l], fmaa(q1, dwx[l], q0 * wx[l]));
  }
}

// Position in a brick's sequence of batches: cell c (0..7; 8 once the sequence is exhausted) and the
// batch's first point b0 within that cell.
struct BrickBatch {
  int c, b0;
};

template <typename A, int OT, int NT, int TSET, bool BUF, bool PAIR>
__global__ __launch_bounds__(64 * BRICK_WAVES) void k_bwd_bricks(CellArgs a) {
  using M = Mfma<A>;
  using Acc = typename M::acc;
  constexpr int BW = 16 * OT;                          // orbitals of a wave
  constexpr int WBW = BRICK_WAVES * BW;                // orbitals of a workgroup
  constexpr int NQ = CELL_PB / 4;                      // steps of four points in a full batch
  constexpr int NB = NT <= 2 ? NT : 5;                 // upstream values per point and orbital tile
  constexpr bool AHEAD = NT <= 2;                      // next batch's upstream values loaded ahead
  constexpr int NBUF = AHEAD ? 2 : 1;                  // batch buffers of upstream values
  constexpr int NQB = AHEAD ? NQ : 1;                  // (more than two terms: none, only one step's)
  // FP32 with the upstream values loaded ahead: the weights of two batches in LDS, so the next
  // batch is staged while the current one is multiplied, with one barrier per batch (an FP64
  // workgroup has no room for the second buffer: two workgroups per CU need under 80 KB each)
  constexpr int NW = (AHEAD && sizeof(A) == 4) ? 2 : 1;
  static_assert(TSET == TSET_ANY || NT == (TSET == TSET_VL || TSET == TSET_VLD ? 2 : (TSET == TSET_V ? 1 : 5)),
                "a fixed term set has its own count");
  static_assert(!PAIR || (OT == 2 && sizeof(A) == 4), "paired orbital columns: FP32, two tiles");
  __shared__ int s_p[2][CELL_PB];                      // point indices of two consecutive batches
  __shared__ A s_w[NW][CELL_PB][36];                   // per point: x, y, z  x  (w[4], w'[4], w''[4])
  __shared__ int s_rng[16];                            // first sorted point and count of the brick's cells
  __shared__ A s_reg[BRICK_ROWS * WBW];                // the brick's region: [row][orbital of the workgroup]
  const int tid = (int)threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int grp = lane >> 4;
  const int col = lane & 15;
  const int m_ = col >> 2, n_ = col & 3;
  // the orbital (within the wave's 16 OT) of the lane's column in orbital tile ot: 16 apart, or with
  // PAIR adjacent (tile ot holds ob + 2 col + ot, so both come in one 8-byte load)
  auto orb_col = [&](int ot) { return PAIR ? 2 * col + ot : ot * 16 + col; };
  const int nbx = (a.g.n[0] + 1) >> 1, nby = (a.g.n[1] + 1) >> 1, nbz = (a.g.n[2] + 1) >> 1;
  const int64_t n_bricks = (int64_t)nbx * nby * nbz;
  const int n_wg = (a.n_groups + BRICK_WAVES - 1) / BRICK_WAVES;   // orbital groups of a workgroup
  const int64_t n_work = n_bricks * n_wg;
  const int nt = TSET == TSET_ANY ? a.n_terms : NT;  // terms in use (a fixed set: a constant)
  const SortedPoint<A>* pts = static_cast<const SortedPoint<A>*>(a.pts);
  A jm[9], mt[6];
#pragma unroll
  for (int i = 0; i < 9; ++i) jm[i] = (A)a.g.jac[i];
#pragma unroll
  for (int i = 0; i < 6; ++i) mt[i] = (A)a.g.metric[i];

  for (int64_t w = blockIdx.x; w < n_work; w += gridDim.x) {
    const int64_t brick = w / n_wg;
    const int obw = (int)(w % n_wg) * WBW;             // first orbital of the workgroup
    const int ob = obw + wave * BW;                    // first orbital of this wave
    const int bz = (int)(brick % nbz);
    const int by = (int)((brick / nbz) % nby);
    const int bx = (int)(brick / ((int64_t)nbz * nby));
    bool ocol[OT];
#pragma unroll
    for (int ot = 0; ot < OT; ++ot) ocol[ot] = ob + orb_col(ot) < a.n_orb;
    __syncthreads();                                   // the previous region is written out
    for (int i = tid; i < BRICK_ROWS * WBW; i += 64 * BRICK_WAVES) s_reg[i] = A(0);
    if (tid < 8) {
      // each cell's sorted point range, bounded like every index read from the workspace
      const int X = 2 * bx + (tid >> 2), Y = 2 * by + ((tid >> 1) & 1), Z = 2 * bz + (tid & 1);
      int start = 0, cnt = 0;
      if (X < a.g.n[0] && Y < a.g.n[1] && Z < a.g.n[2]) {
        const int64_t cell = ((int64_t)X * a.g.n[1] + Y) * a.g.n[2] + Z;
        start = a.cell_range[3 * cell];
        cnt = a.cell_range[3 * cell + 1];
        if (start < 0 || cnt < 0 || start > a.n_pts - cnt) cnt = 0;
      }
      s_rng[tid] = start;
      s_rng[8 + tid] = cnt;
    }
    __syncthreads();
    // lane k (mod 8) holds cell k's range; a wave-uniform cell index reads it with one lane read
    const int lane_start = s_rng[lane & 7], lane_count = s_rng[8 + (lane & 7)];
    auto start_of = [&](int c) { return __builtin_amdgcn_readlane(lane_start, c); };
    auto count_of = [&](int c) { return __builtin_amdgcn_readlane(lane_count, c); };
    auto advance = [&](BrickBatch& b) {
      if (b.c >= 8) return;
      b.b0 += CELL_PB;
      if (b.b0 >= count_of(b.c)) {
        b.b0 = 0;
        ++b.c;
        while (b.c < 8 && count_of(b.c) == 0) ++b.c;
      }
    };
    auto count = [&](const BrickBatch& b) { return b.c < 8 ? min(CELL_PB, count_of(b.c) - b.b0) : 0; };
    // the staging of a batch is shared by 3 CELL_PB threads: thread 3 j + ax holds point j's reduced
    // coordinate on axis ax (and, for ax = 0, its index)
    const int sj = tid / 3, sax = tid - 3 * sj;
    struct Staged {
      A t;
      int p;
    };
    // every thread loads, from an index clamped into the sorted points (threads past the batch
    // discard what they read): a conditional load into these loop-carried registers would make the
    // compiler wait for it at once, where the old and the new value merge
    auto load_points = [&](const BrickBatch& b, Staged& sp) {
      const int64_t k = min(max((int64_t)start_of(min(b.c, 7)) + b.b0 + sj, (int64_t)0), (int64_t)a.n_pts - 1);
      const SortedPoint<A>* rec = pts + k;
      sp.t = rec->t[sax];
      sp.p = rec->p;
    };
    auto stage_index = [&](const BrickBatch& b, const Staged& sp, int* sp_out) {
      if (sax == 0 && sj < count(b)) sp_out[sj] = (unsigned)sp.p < (unsigned)a.n_pts ? sp.p : -1;   // -1: nothing
    };
    auto stage_weights = [&](const BrickBatch& b, const Staged& sp, A (*sw)[36]) {
      if (sj < count(b)) {
        A w4[4], d4[4], dd4[4];
        bspline_weights<A>(sp.t, w4, d4, dd4);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          sw[sj][12 * sax + i] = w4[i];
          sw[sj][12 * sax + 4 + i] = d4[i];
          sw[sj][12 * sax + 8 + i] = dd4[i];
        }
      }
    };
    // upstream values of one step of a batch: lane group k takes point q + k of it.  With BUF (every
    // array under 2 GiB) they are buffer loads with 32-bit byte offsets: the offset of a value is
    // under 2^31, and a dead lane or an orbital past n_orb sets bit 31, which puts the offset beyond
    // the array, so it reads 0 with no branch.
    uint32_t col_off[OT], col_flag[OT];                // byte offset of the lane's orbital in a row
#pragma unroll
    for (int ot = 0; ot < OT; ++ot) {
      col_off[ot] = ocol[ot] ? (uint32_t)(ob + orb_col(ot)) * (uint32_t)sizeof(A) : 0u;
      col_flag[ot] = ocol[ot] ? 0u : 0x80000000u;
    }
    auto load_step = [&](int nb, const int* sp_in, int q, A (&bv)[NB][OT]) {
      const int j = q + grp;
      // -1 past the batch.  With the batch's values loaded ahead (j under CELL_PB), no select of a
      // loaded value, of which the compiler would make a branch; otherwise the next step's j can
      // pass the batch's slots and only the select keeps the read inside them
      int pj;
      if constexpr (AHEAD) pj = sp_in[j] | -(int)(j >= nb);
      else pj = j < nb ? sp_in[j] : -1;
      const bool live = pj >= 0;
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        if (c >= nt) {
#pragma unroll
          for (int ot = 0; ot < OT; ++ot) bv[c][ot] = A(0);
          continue;
        }
        if constexpr (BUF) {
          const __amdgpu_buffer_rsrc_t rs =
              __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(a.src[c]), (short)0, a.src_bytes[c], 0x00020000);
          // ahead: no select on the offset either (the compiler would branch to two loads): a dead
          // lane's pj = -1 carries bit 31 into the offset, whatever the product's low bits
          const uint32_t stride_b = (uint32_t)(a.src_stride[c] * sizeof(A));
          const uint32_t row = AHEAD ? (uint32_t)pj * stride_b : (live ? (uint32_t)pj * stride_b : 0u);
          const uint32_t flag = AHEAD ? ((uint32_t)pj & 0x80000000u) : (live ? 0u : 0x80000000u);
          if constexpr (PAIR) {
            // n_orb is even, so both orbitals of a pair are in range or neither is
            const auto v2 = __builtin_amdgcn_raw_buffer_load_b64(rs, (row + col_off[0]) | flag | col_flag[0], 0, 0);
            bv[c][0] = __uint_as_float(v2[0]);
            bv[c][1] = __uint_as_float(v2[1]);
          } else {
#pragma unroll
            for (int ot = 0; ot < OT; ++ot) bv[c][ot] = BufLoad<A>::load(rs, (row + col_off[ot]) | flag | col_flag[ot]);
          }
        } else {
          const A* src = static_cast<const A*>(a.src[c]);
          const int64_t p = live ? (int64_t)pj : 0;
          if constexpr (PAIR) {
            f2v v2 = f2v{0.0f, 0.0f};
            if (live && ocol[0]) v2 = *reinterpret_cast<const f2v*>(src + p * a.src_stride[c] + ob + orb_col(0));
            bv[c][0] = v2.x;
            bv[c][1] = v2.y;
          } else {
#pragma unroll
            for (int ot = 0; ot < OT; ++ot)
              bv[c][ot] = (live && ocol[ot]) ? src[p * a.src_stride[c] + ob + orb_col(ot)] : A(0);
          }
        }
      }
    };
    auto load_upstream = [&](int nb, const int* sp_in, A (&bv)[NQB][NB][OT]) {
#pragma unroll
      for (int qi = 0; qi < NQB; ++qi) load_step(nb, sp_in, 4 * qi, bv[qi]);
    };
    Acc acc[4][OT];
    // the products of one step of four points: every term's row weights times its upstream values
    auto multiply_step = [&](int nb, int q, const A (*sw)[36], const A (&bv)[NB][OT]) {
      const A* wp = sw[min(q + grp, nb - 1)];         // a dead lane group multiplies zeros
      A wx[4], dwx[4], d2wx[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        wx[i] = wp[i];
        dwx[i] = wp[4 + i];
        d2wx[i] = wp[8 + i];
      }
      const A wy = wp[12 + m_], dwy = wp[16 + m_], d2wy = wp[20 + m_];
      const A wz = wp[24 + n_], dwz = wp[28 + n_], d2wz = wp[32 + n_];
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        if (c >= nt) break;
        const int kind = TSET == TSET_ANY ? a.kind[c]
                                          : (TSET == TSET_VL || TSET == TSET_VLD ? (c == 0 ? TERM_VAL : TERM_LAP) : c);
        A av[4];
        row_weights<A, TSET>(c, kind, wx, dwx, d2wx, wy, dwy, d2wy, wz, dwz, d2wz, jm, mt, av);
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
#pragma unroll
          for (int ot = 0; ot < OT; ++ot) acc[rt][ot] = M::step(av[rt], bv[c][ot], acc[rt][ot]);
      }
    };
    // one batch: with its upstream values already loaded, or (more than two terms) loading each
    // step's values while the step before is multiplied
    auto multiply = [&](int nb, const int* sp_in, const A (*sw)[36], const A (&bv)[NQB][NB][OT]) {
      if constexpr (AHEAD) {
#pragma unroll
        for (int qi = 0; qi < NQB; ++qi)
          if (4 * qi < nb) multiply_step(nb, 4 * qi, sw, bv[qi]);
      } else {
        A bcur[NB][OT];
        load_step(nb, sp_in, 0, bcur);
        for (int q = 0; q < nb; q += 4) {
          // unconditional: past the batch every lane is dead and reads 0 (a conditional load into
          // these loop-carried registers would make the compiler wait for it at once)
          A bnext[NB][OT];
          load_step(nb, sp_in, q + 4, bnext);
          multiply_step(nb, q, sw, bcur);
#pragma unroll
          for (int c = 0; c < NB; ++c)
#pragma unroll
            for (int ot = 0; ot < OT; ++ot) bcur[c][ot] = bnext[c][ot];
        }
      }
    };
    // add the block of cell c into the wave's columns of the region: block row (l, m, n) is region
    // row (cx + l, cy + m, cz + n)
    auto add_block = [&](int c) {
      // region row (cx + l, cy + m, cz + n) = the cell's corner row (uniform) + that of (l, m, n)
      A* corner = s_reg + (((c >> 2) * 5 + ((c >> 1) & 1)) * 5 + (c & 1)) * WBW + wave * BW;
#pragma unroll
      for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int i = M::row(grp, e);
          A* rp = corner + ((rt * 5 + (i >> 2)) * 5 + (i & 3)) * WBW;
#pragma unroll
          for (int ot = 0; ot < OT; ++ot) rp[orb_col(ot)] += acc[rt][ot][e];
        }
    };

    // the first four batches: b0 is multiplied now, b1 is staged, b2 and b3 are in flight
    BrickBatch b0{0, 0};
    while (b0.c < 8 && count_of(b0.c) == 0) ++b0.c;
    BrickBatch b1 = b0;
    advance(b1);
    BrickBatch b2 = b1;
    advance(b2);
    BrickBatch b3 = b2;
    advance(b3);
    Staged sp0, sp_next, sp_after;                     // batches b0, b1 and b2 (used below 3 CELL_PB)
    load_points(b0, sp0);
    load_points(b1, sp_next);
    load_points(b2, sp_after);
    if (tid < 3 * CELL_PB) {
      stage_index(b0, sp0, s_p[0]);
      stage_weights(b0, sp0, s_w[0]);
      stage_index(b1, sp_next, s_p[1]);
    }
    __syncthreads();
    A bq[NBUF][NQB][NB][OT];
    if constexpr (AHEAD) {
      load_upstream(count(b0), s_p[0], bq[0]);
      // every wave has read b0's indices before the first step stages b2's over them
      if constexpr (NW == 2) __syncthreads();
    }
    // one batch: multiply b0, add the block if b0 ends its cell, stage b1's weights and b2's indices,
    // and shift the sequence; `cur` holds b0's upstream values, `nxt` receives b1's
    auto step = [&](int buf, A (&cur)[NQB][NB][OT], A (&nxt)[NQB][NB][OT]) {
      const int nb = count(b0);
      if constexpr (AHEAD) load_upstream(count(b1), s_p[buf ^ 1], nxt);
      if constexpr (NW == 2) {
        // b1's weights go to the other buffer and b2's indices over b0's (b0's upstream values
        // were loaded in the previous step), both while b0 is multiplied
        if (tid < 3 * CELL_PB) {
          stage_weights(b1, sp_next, s_w[buf ^ 1]);
          stage_index(b2, sp_after, s_p[buf]);
        }
        sp_next = sp_after;
        load_points(b3, sp_after);
      }
      if (b0.b0 == 0) {
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
#pragma unroll
          for (int ot = 0; ot < OT; ++ot) acc[rt][ot] = Acc{};
      }
      multiply(nb, s_p[buf], s_w[NW == 2 ? buf : 0], cur);
      if (b0.b0 + CELL_PB >= count_of(b0.c)) add_block(b0.c);
      __syncthreads();                                 // every wave is done with b0's weights and indices
      if constexpr (NW == 1) {
        if (tid < 3 * CELL_PB) {
          stage_weights(b1, sp_next, s_w[0]);
          stage_index(b2, sp_after, s_p[buf]);
        }
        sp_next = sp_after;
        load_points(b3, sp_after);
        __syncthreads();
      }
      b0 = b1;
      b1 = b2;
      b2 = b3;
      advance(b3);
    };
    while (b0.c < 8) {
      step(0, bq[0], bq[NBUF - 1]);
      if (b0.c >= 8) break;
      step(1, bq[NBUF - 1], bq[0]);
    }
    __syncthreads();
    A* out = static_cast<A*>(a.blocks) + brick * BRICK_ROWS * a.o_pad + obw;
    for (int i = tid; i < BRICK_ROWS * WBW; i += 64 * BRICK_WAVES) {
      const int lrow = i / WBW, c = i % WBW;
      if (obw + c < a.n_orb) out[(int64_t)lrow * a.o_pad + c] = s_reg[i];
    }
  }
}

// The region rows that land on table row X along one axis of n rows and nb bricks: region row l
// (0 .. 4) of brick b is row 2 b - 1 + l, taken modulo n.  Each is returned as its share of the
// element offset, b * stride_b + l * stride_l, in a fixed order (images of X from below, bricks
// ascending); at most 3 (a 5-row window moving by 2 covers a row at most 3 times).
__device__ __forceinline__ int brick_parts(int X, int n, int nb, int32_t stride_b, int32_t stride_l, int32_t part[3]) {
  int k = 0;
  for (int img = -1; img <= 1; ++img) {
    const int xp = X + img * n;                        // the row before the wrap
    if (xp < -1 || xp > 2 * nb + 2) continue;
    // 2 b - 1 <= xp <= 2 b + 3  <=>  ceil((xp - 3) / 2) <= b <= floor((xp + 1) / 2)
    const int lo = max((xp - 2) >> 1, 0);              // arithmetic shifts: floor division by 2
    const int hi = min((xp + 1) >> 1, nb - 1);
    for (int b = lo; b <= hi && k < 3; ++b) part[k++] = b * stride_b + (xp - (2 * b - 1)) * stride_l;
  }
  return k;
}

// Dense points, second step: table row (X, Y, Z) receives every brick region row that lands on it
// (at most 3 along each axis), summed in a fixed order and added to the gradient table.  A thread
// takes 16 bytes of orbitals of one row (4 FP32 or 2 FP64 values; the rows are padded to 16 bytes),
// so a wave covers whole rows with 16-byte loads; the offset of a region row is the sum of its
// three axis shares, and every region row is loaded before the sum, so the loads are in flight
// together.  Each orbital's sum runs over the region rows in the same order whatever the vector
// width.  Orbitals of the row's padding are read from the regions and summed, but the gradient
// table's padding is never touched.
constexpr int GATHER_MAX = 27;

template <typename A>
__global__ __launch_bounds__(256) void k_bwd_brick_gather(Geom g, const A* regions, int32_t n_orb, int32_t o_pad,
                                                          int32_t per_row, int64_t n_rows, A* gtab) {
  constexpr int V = 16 / (int)sizeof(A);
  typedef A Vec __attribute__((ext_vector_type(V)));
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t row = idx / per_row;
  if (row >= n_rows) return;
  const int o = (int)(idx - row * per_row) * V;        // first orbital of the thread
  const int Z = (int)(row % g.n[2]);
  const int Y = (int)((row / g.n[2]) % g.n[1]);
  const int X = (int)(row / ((int64_t)g.n[2] * g.n[1]));
  const int nbx = (g.n[0] + 1) >> 1, nby = (g.n[1] + 1) >> 1, nbz = (g.n[2] + 1) >> 1;
  // element offsets fit in 32 bits: the regions are capped at 4 GiB
  const int32_t sz = BRICK_ROWS * o_pad, sy = nbz * sz, sx = nby * sy;
  int32_t px[3], py[3], pz[3];
  const int kx = brick_parts(X, g.n[0], nbx, sx, 25 * o_pad, px);
  const int ky = brick_parts(Y, g.n[1], nby, sy, 5 * o_pad, py);
  const int kz = brick_parts(Z, g.n[2], nbz, sz, o_pad, pz);
  Vec part[GATHER_MAX];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const bool live = i < kx && j < ky && k < kz;
        part[9 * i + 3 * j + k] =
            live ? *reinterpret_cast<const Vec*>(regions + (int64_t)(px[i] + py[j] + pz[k]) + o) : Vec(0);
      }
  Vec sum = Vec(0);
#pragma unroll
  for (int c = 0; c < GATHER_MAX; ++c) sum += part[c];
  A* dst = gtab + row * o_pad + o;
  if (o + V <= n_orb) {
    Vec cur = *reinterpret_cast<Vec*>(dst);
    cur += sum;
    *reinterpret_cast<Vec*>(dst) = cur;
  } else {
    // the row's last orbitals: the padding columns are neither read nor written
#pragma unroll
    for (int v = 0; v < V; ++v)
      if (o + v < n_orb) dst[v] += sum[v];
  }
}

// the gather over every table row: 16 bytes of orbitals per thread
template <typename A>
static int launch_brick_gather(const spl_desc* d, const Geom& g, const void* regions, void* gtable, hipStream_t stream) {
  constexpr int V = 16 / (int)sizeof(A);
  const int per_row = (d->n_orb + V - 1) / V;          // within the padded row: o_pad is a multiple of V
  const int64_t n_rows = (int64_t)d->grid[0] * d->grid[1] * d->grid[2];
  const int64_t blocks = (n_rows * per_row + 255) / 256;
  hipLaunchKernelGGL(k_bwd_brick_gather<A>, dim3((unsigned)blocks), dim3(256), 0, stream, g,
                     static_cast<const A*>(regions), d->n_orb, d->o_pad, (int32_t)per_row, n_rows, static_cast<A*>(gtable));
  return hip_fail(hipGetLastError(), "row gather launch");
}

// Sparse points (fewer than 2.5 per cell on average): the gradient formed row-tile by row-tile.  Along
// an axis a point of cell i touches rows i - 1 .. i + 2 (Eq. b-splineapproximation), so row X
// receives the points of cells X - 2 .. X + 1, and a tile of 4 x 4 x 4 rows those of a window of
// 7 x 7 x 7 cells (the whole axis when it has fewer than 7 cells; the last tile of an axis holds
// its last N mod 4 rows, or 4).  One workgroup per (tile, group of TILE_WAVES x 16 OT orbitals)
// forms the tile's gradient as one dense product on the matrix cores,
//     d beta[row][o] = sum over the window's points and the terms of W_term(point)[row] g_term[point][o],
// where a point's 1-D weights are moved onto the tile rows they land on (0 on a tile row outside
// its support), and adds it to the table once.  Every row belongs to one workgroup: no atomics,
// one launch, and a fixed order of every sum (window cells in order, each cell's points in sorted
// order).  Each point is multiplied with the whole tile, so the matrix cores do about (7/4)^3 times
// the useful products; with under 2.5 points per cell that costs less than a workspace region per
// brick, which would be read and written for few points.
//
// The window's points are taken in batches of CELL_PB across cell boundaries (slot q of the window
// is found by a binary search over the prefix sums of its cells' counts): the records of later
// batches load while the current batch is multiplied, their weights and indices are staged in a
// second LDS buffer, and each step's upstream values load while the step before is multiplied.
// A window holds few batches (about 7 on the Si-like cell, 1 on the MgO-like cell), so what hides
// its chain of dependent accesses is the number of workgroups in flight: the kernel is held to 3
// waves per SIMD (measured: loading a whole batch's upstream values ahead, in registers that allow
// only 2, was 8-27% slower).
constexpr int TILE_WAVES = 4;
constexpr int TILE_WIN = 7;                               // window cells per axis (at most)
constexpr int TILE_WIN3 = TILE_WIN * TILE_WIN * TILE_WIN;

template <typename A>
__device__ __forceinline__ A select4(int l, A a0, A a1, A a2, A a3) {
  return l == 0 ? a0 : (l == 1 ? a1 : (l == 2 ? a2 : a3));
}

template <typename A, int OT, int NT, int TSET, bool BUF>
__global__ __launch_bounds__(64 * TILE_WAVES) __attribute__((amdgpu_waves_per_eu(3))) void k_bwd_tiles(CellArgs a) {
  using M = Mfma<A>;
  using Acc = typename M::acc;
  constexpr int BW = 16 * OT;                          // orbitals of a wave
  constexpr int WBW = TILE_WAVES * BW;                 // orbitals of a workgroup
  constexpr int NB = NT <= 2 ? NT : 5;                 // upstream values per point and orbital tile
  static_assert(2 * 64 * TILE_WAVES >= TILE_WIN3, "two window cells per thread");
  static_assert(TSET == TSET_ANY || NT == (TSET == TSET_VL || TSET == TSET_VLD ? 2 : (TSET == TSET_V ? 1 : 5)),
                "a fixed term set has its own count");
  __shared__ int s_start[TILE_WIN3];                   // first sorted point of each window cell
  __shared__ int s_pre[TILE_WIN3 + 1];                 // points of the window cells before each
  __shared__ int s_wsum[TILE_WAVES];
  __shared__ int s_p[2][CELL_PB];                      // point indices of two consecutive batches
  __shared__ A s_w[2][CELL_PB][36];                    // per point: x, y, z  x  tile rows of (w, w', w'')
  const int tid = (int)threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int grp = lane >> 4;
  const int col = lane & 15;
  const int m_ = col >> 2, n_ = col & 3;
  const int nt_x = (a.g.n[0] + 3) >> 2, nt_y = (a.g.n[1] + 3) >> 2, nt_z = (a.g.n[2] + 3) >> 2;
  const int64_t n_tiles = (int64_t)nt_x * nt_y * nt_z;
  const int n_wg = (a.n_groups + TILE_WAVES - 1) / TILE_WAVES;
  const int64_t n_work = n_tiles * n_wg;
  const int nw[3] = {min(a.g.n[0], TILE_WIN), min(a.g.n[1], TILE_WIN), min(a.g.n[2], TILE_WIN)};
  const int nwin = nw[0] * nw[1] * nw[2];
  const int nt = TSET == TSET_ANY ? a.n_terms : NT;
  const SortedPoint<A>* pts = static_cast<const SortedPoint<A>*>(a.pts);
  A* gtab = static_cast<A*>(a.gtable);
  A jm[9], mt[6];
#pragma unroll
  for (int i = 0; i < 9; ++i) jm[i] = (A)a.g.jac[i];
#pragma unroll
  for (int i = 0; i < 6; ++i) mt[i] = (A)a.g.metric[i];

  for (int64_t w = blockIdx.x; w < n_work; w += gridDim.x) {
    const int64_t tile = w / n_wg;
    const int ob = (int)(w % n_wg) * WBW + wave * BW;  // first orbital of this wave
    const int x0[3] = {4 * (int)(tile / ((int64_t)nt_z * nt_y)), 4 * (int)((tile / nt_z) % nt_y),
                       4 * (int)(tile % nt_z)};
    // window cell k along axis ax: cell x0 - 2 + k (mod N), or cell k of an axis under 7 cells
    auto win_cell = [&](int ax, int k) {
      if (a.g.n[ax] < TILE_WIN) return k;
      const int c = x0[ax] - 2 + k;
      return c < 0 ? c + a.g.n[ax] : (c >= a.g.n[ax] ? c - a.g.n[ax] : c);
    };
    bool ocol[OT];
#pragma unroll
    for (int ot = 0; ot < OT; ++ot) ocol[ot] = ob + ot * 16 + col < a.n_orb;
    __syncthreads();                                   // the previous tile is done with the LDS
    // the window cells' point ranges (thread t: cells 2t and 2t + 1), bounded like every index read
    // from the workspace, and the exclusive prefix of their counts
    int cnt2[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int c = 2 * tid + h;
      cnt2[h] = 0;
      if (c < nwin) {
        const int kz = c % nw[2], ky = (c / nw[2]) % nw[1], kx = c / (nw[2] * nw[1]);
        const int64_t cell = ((int64_t)win_cell(0, kx) * a.g.n[1] + win_cell(1, ky)) * a.g.n[2] + win_cell(2, kz);
        int start = a.cell_range[3 * cell], cnt = a.cell_range[3 * cell + 1];
        if (start < 0 || cnt < 0 || start > a.n_pts - cnt) start = cnt = 0;
        s_start[c] = start;
        cnt2[h] = cnt;
      }
    }
    const int mine = cnt2[0] + cnt2[1];
    int incl = mine;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int up = __shfl_up(incl, d);
      if (lane >= d) incl += up;
    }
    if (lane == 63) s_wsum[wave] = incl;
    __syncthreads();
    int before = 0;
    for (int v = 0; v < wave; ++v) before += s_wsum[v];
    const int excl = before + incl - mine;
    if (2 * tid < nwin) s_pre[2 * tid] = excl;
    if (2 * tid + 1 < nwin) s_pre[2 * tid + 1] = excl + cnt2[0];
    if (2 * tid < nwin && 2 * tid + 2 >= nwin) s_pre[nwin] = excl + mine;
    __syncthreads();
    const int total = s_pre[nwin];
    if (total == 0) continue;                          // no point reaches this tile: its rows stay as they are
    const int n_bat = (total + CELL_PB - 1) / CELL_PB;
    auto count = [&](int k) { return k < n_bat ? min(CELL_PB, total - k * CELL_PB) : 0; };

    // the staging of a batch is shared by 3 CELL_PB threads: thread 3 j + ax holds point j's
    // reduced coordinate and cell on axis ax (and, for ax = 0, its index)
    const int sj = tid / 3, sax = tid - 3 * sj;
    struct Staged {
      A t;
      int p, cell;
    };
    // every thread loads (slot clamped into the window, so threads past the batch read a real record)
    auto load_points = [&](int k, Staged& sp) {
      const int q = (int)min((int64_t)k * CELL_PB + sj, (int64_t)total - 1);
      int lo = 0, hi = nwin;                           // s_pre[lo] <= q < s_pre[hi]
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (s_pre[mid] <= q) lo = mid;
        else hi = mid;
      }
      const int s = min(max(s_start[lo] + q - s_pre[lo], 0), a.n_pts - 1);
      const SortedPoint<A>* rec = pts + s;
      sp.t = rec->t[sax];
      sp.p = rec->p;
      const int k_ax = sax == 0 ? lo / (nw[2] * nw[1]) : (sax == 1 ? (lo / nw[2]) % nw[1] : lo % nw[2]);
      sp.cell = win_cell(sax, k_ax);
    };
    auto stage_index = [&](int k, const Staged& sp, int* sp_out) {
      if (sax == 0 && sj < count(k)) sp_out[sj] = (unsigned)sp.p < (unsigned)a.n_pts ? sp.p : -1;
    };
    // tile row x0 + r lies at offset l = x0 + r - (cell - 1) (mod N) of the point's support; its weight
    // is w[l] for l <= 3 and 0 otherwise
    auto stage_weights = [&](int k, const Staged& sp, A (*sw)[36]) {
      if (sj < count(k)) {
        A w4[4], d4[4], dd4[4];
        bspline_weights<A>(sp.t, w4, d4, dd4);
        const int n = a.g.n[sax];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          int l = x0[sax] + r - sp.cell + 1;
          l = l < 0 ? l + n : (l >= n ? l - n : l);
          const bool in = l <= 3;
          sw[sj][12 * sax + r] = in ? select4(l, w4[0], w4[1], w4[2], w4[3]) : A(0);
          sw[sj][12 * sax + 4 + r] = in ? select4(l, d4[0], d4[1], d4[2], d4[3]) : A(0);
          sw[sj][12 * sax + 8 + r] = in ? select4(l, dd4[0], dd4[1], dd4[2], dd4[3]) : A(0);
        }
      }
    };
    uint32_t col_off[OT], col_flag[OT];                // byte offset of the lane's orbital in a row
#pragma unroll
    for (int ot = 0; ot < OT; ++ot) {
      col_off[ot] = ocol[ot] ? (uint32_t)(ob + ot * 16 + col) * (uint32_t)sizeof(A) : 0u;
      col_flag[ot] = ocol[ot] ? 0u : 0x80000000u;
    }
    // upstream values of one step of a batch (as in the brick kernel): lane group k takes point q + k
    auto load_step = [&](int nb, const int* sp_in, int q, A (&bv)[NB][OT]) {
      const int j = q + grp;
      const int pj = j < nb ? sp_in[j] : -1;
      const bool live = pj >= 0;
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        if (c >= nt) {
#pragma unroll
          for (int ot = 0; ot < OT; ++ot) bv[c][ot] = A(0);
          continue;
        }
        if constexpr (BUF) {
          const __amdgpu_buffer_rsrc_t rs =
              __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(a.src[c]), (short)0, a.src_bytes[c], 0x00020000);
          const uint32_t row = live ? (uint32_t)pj * (uint32_t)(a.src_stride[c] * sizeof(A)) : 0u;
          const uint32_t flag = live ? 0u : 0x80000000u;
#pragma unroll
          for (int ot = 0; ot < OT; ++ot) bv[c][ot] = BufLoad<A>::load(rs, (row + col_off[ot]) | flag | col_flag[ot]);
        } else {
          const A* src = static_cast<const A*>(a.src[c]);
          const int64_t p = live ? (int64_t)pj : 0;
#pragma unroll
          for (int ot = 0; ot < OT; ++ot)
            bv[c][ot] = (live && ocol[ot]) ? src[p * a.src_stride[c] + ob + ot * 16 + col] : A(0);
        }
      }
    };
    Acc acc[4][OT];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
      for (int ot = 0; ot < OT; ++ot) acc[rt][ot] = Acc{};
    // the products of one step of four points (as in the brick kernel, on tile rows)
    auto multiply_step = [&](int nb, int q, const A (*sw)[36], const A (&bv)[NB][OT]) {
      const A* wp = sw[min(q + grp, nb - 1)];         // a dead lane group multiplies zeros
      A wx[4], dwx[4], d2wx[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        wx[i] = wp[i];
        dwx[i] = wp[4 + i];
        d2wx[i] = wp[8 + i];
      }
      const A wy = wp[12 + m_], dwy = wp[16 + m_], d2wy = wp[20 + m_];
      const A wz = wp[24 + n_], dwz = wp[28 + n_], d2wz = wp[32 + n_];
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        if (c >= nt) break;
        const int kind = TSET == TSET_ANY ? a.kind[c]
                                          : (TSET == TSET_VL || TSET == TSET_VLD ? (c == 0 ? TERM_VAL : TERM_LAP) : c);
        A av[4];
        row_weights<A, TSET>(c, kind, wx, dwx, d2wx, wy, dwy, d2wy, wz, dwz, d2wz, jm, mt, av);
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
#pragma unroll
          for (int ot = 0; ot < OT; ++ot) acc[rt][ot] = M::step(av[rt], bv[c][ot], acc[rt][ot]);
      }
    };
    // one batch: each step's upstream values load while the step before is multiplied
    auto multiply = [&](int nb, const int* sp_in, const A (*sw)[36]) {
      A bcur[NB][OT];
      load_step(nb, sp_in, 0, bcur);
      for (int q = 0; q < nb; q += 4) {
        A bnext[NB][OT];                               // unconditional: past the batch every lane reads 0
        load_step(nb, sp_in, q + 4, bnext);
        multiply_step(nb, q, sw, bcur);
#pragma unroll
        for (int c = 0; c < NB; ++c)
#pragma unroll
          for (int ot = 0; ot < OT; ++ot) bcur[c][ot] = bnext[c][ot];
      }
    };

    // batch 0 is multiplied first, batch 1 is staged, batch 2's record is in flight
    Staged sp0, sp_next, sp_after;
    load_points(0, sp0);
    load_points(1, sp_next);
    load_points(2, sp_after);
    if (tid < 3 * CELL_PB) {
      stage_index(0, sp0, s_p[0]);
      stage_weights(0, sp0, s_w[0]);
      stage_index(1, sp_next, s_p[1]);
    }
    __syncthreads();
    // batch k: stage batch k + 1's weights, multiply batch k, then (every wave done with batch k's
    // indices) stage batch k + 2's indices over them
    for (int k = 0; k < n_bat; ++k) {
      const int buf = k & 1;
      if (tid < 3 * CELL_PB) stage_weights(k + 1, sp_next, s_w[buf ^ 1]);
      multiply(count(k), s_p[buf], s_w[buf]);
      __syncthreads();                                 // every wave is done with batch k's weights and indices
      if (tid < 3 * CELL_PB) stage_index(k + 2, sp_after, s_p[buf]);
      sp_next = sp_after;
      load_points(k + 3, sp_after);
    }
    // the tile's rows inside the table: every old value is loaded before the first store
    A old[4][4][OT];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = M::row(grp, e);                  // 4 m + n within the row tile
        const int X = x0[0] + rt, Y = x0[1] + (i >> 2), Z = x0[2] + (i & 3);
        const bool in = X < a.g.n[0] && Y < a.g.n[1] && Z < a.g.n[2];
        const A* rp = gtab + (int64_t)X * a.g.s0 + (int64_t)Y * a.g.s1 + (int64_t)Z * a.g.o_pad + ob + col;
#pragma unroll
        for (int ot = 0; ot < OT; ++ot) old[rt][e][ot] = (in && ocol[ot]) ? rp[16 * ot] : A(0);
      }
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = M::row(grp, e);
        const int X = x0[0] + rt, Y = x0[1] + (i >> 2), Z = x0[2] + (i & 3);
        const bool in = X < a.g.n[0] && Y < a.g.n[1] && Z < a.g.n[2];
        A* rp = gtab + (int64_t)X * a.g.s0 + (int64_t)Y * a.g.s1 + (int64_t)Z * a.g.o_pad + ob + col;
#pragma unroll
        for (int ot = 0; ot < OT; ++ot)
          if (in && ocol[ot]) rp[16 * ot] = old[rt][e][ot] + acc[rt][ot][e];
      }
  }
}

// Each occupied cell's sorted point range (first point, count) and run index; the runs past the
// finite points' (the non-finite points' sentinel key) are left out.
__global__ void k_cell_ranges(const int64_t* uniq, const int32_t* counts, const int32_t* offsets,
                              const int32_t* finite_runs, int64_t n_cells, int32_t n_pts, int32_t* cell_range) {
  const int n_runs = (int)min((int64_t)min(max(*finite_runs, 0), n_pts), n_cells);
  const int r = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (r >= n_runs) return;
  const int64_t cell = uniq[r] % n_cells;
  if (cell >= 0) {
    cell_range[3 * cell] = offsets[r];
    cell_range[3 * cell + 1] = counts[r];
    cell_range[3 * cell + 2] = r;
  }
}

__global__ void k_bwd_fill_i32(int32_t* p, int64_t n, int32_t value) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = value;
}

typedef void (*CellKernel)(CellArgs);

// brick regions: FP32 two orbital tiles per wave, FP64 one (64 KB of LDS for a workgroup's region either way)
template <typename A, bool BUF, bool PAIR>
static CellKernel pick_bricks_buf(int nt, int tset) {
  constexpr int OT = sizeof(A) == 4 ? 2 : 1;
  if (tset == TSET_V) return k_bwd_bricks<A, OT, 1, TSET_V, BUF, PAIR>;
  if (tset == TSET_VL) return k_bwd_bricks<A, OT, 2, TSET_VL, BUF, PAIR>;
  if (tset == TSET_VLD) return k_bwd_bricks<A, OT, 2, TSET_VLD, BUF, PAIR>;
  if (tset == TSET_ALLD) return k_bwd_bricks<A, OT, 5, TSET_ALLD, BUF, PAIR>;
  if (tset == TSET_ALL) return k_bwd_bricks<A, OT, 5, TSET_ALL, BUF, PAIR>;
  return nt <= 2 ? k_bwd_bricks<A, OT, 2, TSET_ANY, BUF, PAIR> : k_bwd_bricks<A, OT, 5, TSET_ANY, BUF, PAIR>;
}
// pair: FP32 with an even orbital count and 8-byte aligned upstream arrays; tset as for the row tiles
template <typename A>
static CellKernel pick_bricks(int nt, int tset, bool buf, bool pair) {
  if constexpr (sizeof(A) == 4) {
    if (pair) return buf ? pick_bricks_buf<A, true, true>(nt, tset) : pick_bricks_buf<A, false, true>(nt, tset);
  }
  return buf ? pick_bricks_buf<A, true, false>(nt, tset) : pick_bricks_buf<A, false, false>(nt, tset);
}
template <typename A>
static int brick_ot() {
  return sizeof(A) == 4 ? 2 : 1;
}

// row tiles: the orbital tiles of the brick form; tset: a fixed term set (TSET_V, TSET_VL, TSET_VLD, TSET_ALL,
// TSET_ALLD) where the terms are that set
template <typename A, bool BUF>
static CellKernel pick_tiles_buf(int nt, int tset) {
  constexpr int OT = sizeof(A) == 4 ? 2 : 1;
  if (tset == TSET_V) return k_bwd_tiles<A, OT, 1, TSET_V, BUF>;
  if (tset == TSET_VL) return k_bwd_tiles<A, OT, 2, TSET_VL, BUF>;
  if (tset == TSET_VLD) return k_bwd_tiles<A, OT, 2, TSET_VLD, BUF>;
  if (tset == TSET_ALLD) return k_bwd_tiles<A, OT, 5, TSET_ALLD, BUF>;
  if (tset == TSET_ALL) return k_bwd_tiles<A, OT, 5, TSET_ALL, BUF>;
  return nt <= 2 ? k_bwd_tiles<A, OT, 2, TSET_ANY, BUF> : k_bwd_tiles<A, OT, 5, TSET_ANY, BUF>;
}
template <typename A>
static CellKernel pick_tiles(int nt, int tset, bool buf) {
  return buf ? pick_tiles_buf<A, true>(nt, tset) : pick_tiles_buf<A, false>(nt, tset);
}

// The points sorted by cell: keys, permutation, runs of one cell with their point ranges, the number
// of runs of finite points, and each sorted point's record.
struct CellSort {
  int64_t* keys;         // sorted keys (the cell; non-finite points: n_cells, last)
  int32_t* perm;         // sorted position -> point index
  int64_t* uniq;         // key of each run
  int32_t* counts;       // points in each run
  int32_t* offsets;      // first sorted position of each run
  int32_t* finite_runs;  // runs of finite points (one value)
  void* pts;             // SortedPoint records in sorted order
  char* base;            // the workspace
};

// The sort's arrays in a workspace laid out by L (no kernels run).
static CellSort cell_sort_view(void* work, const SortLayout& L) {
  char* W = static_cast<char*>(work);
  return CellSort{reinterpret_cast<int64_t*>(W + L.keys_out), reinterpret_cast<int32_t*>(W + L.vals_out),
                  reinterpret_cast<int64_t*>(W + L.uniq), reinterpret_cast<int32_t*>(W + L.counts),
                  reinterpret_cast<int32_t*>(W + L.offsets), reinterpret_cast<int32_t*>(W + L.finite_runs),
                  W + L.pts, W};
}

// Sorts the points into the workspace (or, with reuse, takes the sort an earlier call left there).
static int cell_sort(const spl_desc* d, int64_t n_pts, const double* pos, void* work, const SortLayout& L,
                     bool reuse, hipStream_t stream, CellSort* cs) {
  if (reuse) {
    *cs = cell_sort_view(work, L);
    return SPL_OK;
  }
  int rc;
  char* W = static_cast<char*>(work);
  int64_t* keys_in = reinterpret_cast<int64_t*>(W + L.keys_in);
  int64_t* keys_out = reinterpret_cast<int64_t*>(W + L.keys_out);
  int32_t* vals_in = reinterpret_cast<int32_t*>(W + L.vals_in);
  int32_t* vals_out = reinterpret_cast<int32_t*>(W + L.vals_out);
  int64_t* uniq = reinterpret_cast<int64_t*>(W + L.uniq);
  int32_t* counts = reinterpret_cast<int32_t*>(W + L.counts);
  int32_t* offsets = reinterpret_cast<int32_t*>(W + L.offsets);
  int32_t* num_runs = reinterpret_cast<int32_t*>(W + L.num_runs);
  int32_t* finite_runs = reinterpret_cast<int32_t*>(W + L.finite_runs);
  void* pts = W + L.pts;
  void* temp = W + L.temp;
  const Geom g = make_geom(d);
  const int n = (int)n_pts;
  hipLaunchKernelGGL(k_cell_keys, dim3((n + 255) / 256), dim3(256), 0, stream, g, pos, (int32_t)n, L.n_cells,
                     L.n_cells, keys_in, vals_in);
  if ((rc = hip_fail(hipGetLastError(), "cell key launch"))) return rc;
  size_t tb = L.temp_bytes;
  if ((rc = hip_fail(sort_cell_keys(temp, tb, keys_in, keys_out, vals_in, vals_out, n, L.end_bit, stream),
                     "radix sort")))
    return rc;
  tb = L.temp_bytes;
  if ((rc = hip_fail(hipcub::DeviceRunLengthEncode::Encode(temp, tb, keys_out, uniq, counts, num_runs, n, stream),
                     "run-length encode")))
    return rc;
  tb = L.temp_bytes;
  if ((rc = hip_fail(hipcub::DeviceScan::ExclusiveSum(temp, tb, counts, offsets, n, stream), "scan"))) return rc;
  hipLaunchKernelGGL(k_finite_runs, dim3(1), dim3(64), 0, stream, uniq, num_runs, L.n_cells, finite_runs);
  if ((rc = hip_fail(hipGetLastError(), "class start launch"))) return rc;
  if (d->dtype == SPL_F64)
    hipLaunchKernelGGL(k_sorted_points<double>, dim3((n + 255) / 256), dim3(256), 0, stream, g, pos, vals_out,
                       (int32_t)n, static_cast<SortedPoint<double>*>(pts));
  else
    hipLaunchKernelGGL(k_sorted_points<float>, dim3((n + 255) / 256), dim3(256), 0, stream, g, pos, vals_out,
                       (int32_t)n, static_cast<SortedPoint<float>*>(pts));
  if ((rc = hip_fail(hipGetLastError(), "sorted point launch"))) return rc;

  *cs = cell_sort_view(work, L);
  return SPL_OK;
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
                           const void* glap, void* gtable, void* work, int64_t work_bytes, bool reuse,
                           hipStream_t stream) {
  if (n_pts == 0 || !gtable) return SPL_OK;
  SortLayout L;
  int rc = sort_layout(d, n_pts, &L);
  if (rc) return rc;
  if (!work || work_bytes < (int64_t)L.total)
    return fail(SPL_EINVAL, "deterministic backward needs a workspace of %lld bytes", (long long)L.total);
  CellSort cs;
  if ((rc = cell_sort(d, n_pts, pos, work, L, reuse, stream, &cs))) return rc;
  char* W = cs.base;
  int64_t* uniq = cs.uniq;
  int32_t* counts = cs.counts;
  int32_t* offsets = cs.offsets;
  void* pts = cs.pts;
  const Geom g = make_geom(d);

  // orbital tiles of 16 per wave: FP32 two, FP64 one (brick and row-tile forms alike)
  const int tiles = (d->n_orb + 15) / 16;
  const int ot = d->dtype == SPL_F64 ? brick_ot<double>() : brick_ot<float>();
  CellArgs a;
  memset(&a, 0, sizeof(a));
  a.g = g;
  a.pos = pos;
  a.pts = pts;
  a.n_cells = L.n_cells;
  a.n_orb = d->n_orb;
  a.n_groups = (tiles + ot - 1) / ot;
  a.n_pts = (int32_t)n_pts;
  a.o_pad = d->o_pad;
  {
    // each cell's sorted point range (empty cells: none), from the sort
    int32_t* cell_range = reinterpret_cast<int32_t*>(W + L.cell_range);
    if (L.dense) a.blocks = W + L.blocks;
    a.cell_range = cell_range;
    hipLaunchKernelGGL(k_bwd_fill_i32, dim3((unsigned)((3 * L.n_cells + 255) / 256)), dim3(256), 0, stream,
                       cell_range, 3 * L.n_cells, 0);
    if ((rc = hip_fail(hipGetLastError(), "cell range clear launch"))) return rc;
    const int max_runs = (int)std::min<int64_t>(n_pts, L.n_cells);
    hipLaunchKernelGGL(k_cell_ranges, dim3((unsigned)((max_runs + 255) / 256)), dim3(256), 0, stream, uniq, counts,
                       offsets, cs.finite_runs, L.n_cells, (int32_t)n_pts, cell_range);
    if ((rc = hip_fail(hipGetLastError(), "cell range launch"))) return rc;
  }
  const int64_t no = d->n_orb;
  const size_t gsz = d->dtype == SPL_F64 ? 8 : 4;
  const int passes = d->has_lap ? 2 : 1;
  for (int pass = 0; pass < passes; ++pass) {
    // pass 0: the orbital table (value, gradient, and the Laplacian unless it has its own table);
    // pass 1: the separate Laplacian table, whose rows carry the value weights of gL
    int nt = 0;
    auto term = [&](const void* src, int64_t stride, int kind) {
      a.src[nt] = src;
      a.src_stride[nt] = stride;
      a.kind[nt] = kind;
      ++nt;
    };
    if (pass == 0) {
      if (gv) term(gv, no, TERM_VAL);
      if (ggrad) {
        const char* gb = static_cast<const char*>(ggrad);
        term(gb, 3 * no, TERM_GX);
        term(gb + no * gsz, 3 * no, TERM_GY);
        term(gb + 2 * no * gsz, 3 * no, TERM_GZ);
      }
      if (glap && !d->has_lap) term(glap, no, TERM_LAP);
    } else if (glap) {
      term(glap, no, TERM_VAL);
    }
    if (nt == 0) continue;
    a.n_terms = nt;
    for (int c = 0; c < 5; ++c) {
      // from src[c] to the last point's last orbital
      const int64_t bytes = c < nt ? ((int64_t)(n_pts - 1) * a.src_stride[c] + no) * (int64_t)gsz : 0;
      a.src_bytes[c] = bytes < ((int64_t)1 << 31) - 4096 ? (int32_t)bytes : -1;
    }
    a.gtable = static_cast<char*>(gtable) + (pass == 1 ? d->table_elems * gsz : 0);
    bool buf = true, pair = d->n_orb % 2 == 0;
    for (int c = 0; c < nt; ++c) {
      buf = buf && a.src_bytes[c] >= 0;
      pair = pair && a.src_stride[c] % 2 == 0 && reinterpret_cast<uintptr_t>(a.src[c]) % 8 == 0;
    }
    // a term set the kernels fix at compile time: the value alone, the fit's pair, all five in order
    bool all = nt == 5;
    for (int c = 0; c < nt; ++c) all = all && a.kind[c] == TERM_VAL + c;
    const bool vl = nt == 2 && a.kind[0] == TERM_VAL && a.kind[1] == TERM_LAP;
    const DiagForms df = diag_forms(d);
    const int tset = vl ? (df.diag ? TSET_VLD : TSET_VL)
                        : (all ? (df.diag_jac ? TSET_ALLD : TSET_ALL)
                               : (nt == 1 && a.kind[0] == TERM_VAL ? TSET_V : TSET_ANY));
    if (L.dense) {
      // every brick at once into its region, then one gather per table row
      const CellKernel kb = d->dtype == SPL_F64 ? pick_bricks<double>(nt, tset, buf, false)
                                                : pick_bricks<float>(nt, tset, buf, pair);
      const int64_t n_bricks = (int64_t)((d->grid[0] + 1) / 2) * ((d->grid[1] + 1) / 2) * ((d->grid[2] + 1) / 2);
      const int64_t n_wg = (a.n_groups + BRICK_WAVES - 1) / BRICK_WAVES;
      const int grid = (int)std::min<int64_t>(n_bricks * n_wg, 1 << 16);
      hipLaunchKernelGGL(kb, dim3(grid), dim3(64 * BRICK_WAVES), 0, stream, a);
      if ((rc = hip_fail(hipGetLastError(), "brick region launch"))) return rc;
      rc = d->dtype == SPL_F64 ? launch_brick_gather<double>(d, g, a.blocks, a.gtable, stream)
                               : launch_brick_gather<float>(d, g, a.blocks, a.gtable, stream);
      if (rc) return rc;
      continue;
    }
    // sparse points: every tile of 4 x 4 x 4 rows at once, each from its window of cells
    const CellKernel kt = d->dtype == SPL_F64 ? pick_tiles<double>(nt, tset, buf) : pick_tiles<float>(nt, tset, buf);
    const int64_t n_tiles = (int64_t)((d->grid[0] + 3) / 4) * ((d->grid[1] + 3) / 4) * ((d->grid[2] + 3) / 4);
    const int64_t n_wg = (a.n_groups + TILE_WAVES - 1) / TILE_WAVES;
    const int grid = (int)std::min<int64_t>(n_tiles * n_wg, 1 << 16);
    hipLaunchKernelGGL(kt, dim3(grid), dim3(64 * TILE_WAVES), 0, stream, a);
    if ((rc = hip_fail(hipGetLastError(), "row tile launch"))) return rc;
  }
  return SPL_OK;
}


// ---------------------------------------------------------------------------------------------
// Forward evaluation cell by cell (spline_eval_vgl_cells).  For the points of one cell the
// outputs are a dense product: out_term[point][o] = sum over the 64 rows of the cell's block of
// W_term(point)[row] beta[row][o] (Eq. b-splineapproximation with the chain rule of Sec. II), so
// a wave loads the block once, as matrix-core B operands (k-step ks covers rows 4 ks .. 4 ks + 3:
// block offsets l = ks / 4, m = ks mod 4 and n = the lane group), and multiplies it with the row
// weights of up to 32 of the cell's points (two M tiles of 16) per batch.  Where points are
// dense each block row is read once per cell instead of once per point.

struct FwdArgs {
  Geom g;
  const void* table;       // orbital table; the Laplacian table follows at lap_off elements
  int64_t lap_off;
  void* out[5];            // output base of each term (point-major)
  int64_t out_stride[5];   // elements from one point to the next
  int32_t kind[5];         // TERM_* of each term (TERM_VAL of the Laplacian table for a separate one)
  int32_t src[5];          // 0: the orbital table, 1: the Laplacian table
  int32_t n_terms;
  int32_t use_lap_table;
  const int64_t* uniq;
  const int32_t* counts;
  const int32_t* offsets;
  const void* pts;
  const int32_t* finite_runs;  // runs of finite points (occupied cells), from the sort
  int64_t n_cells;
  int32_t n_orb;
  int32_t n_groups;
  int32_t n_pts;           // every index read from the sort is checked against this and n_cells
  // fit terms (spline_fit_terms_cells): a term with a target writes 2 w (y - t) instead of y and
  // adds w (y - t)^2 to its work item's FP64 partial sum
  const void* target[5];
  double w[5];
  double* partial;         // one slot per work item (NULL: plain outputs)
};

template <typename TS> struct Stored;
template <> struct Stored<double> {
  __device__ __forceinline__ static double at(const double* p) { return *p; }
};
template <> struct Stored<float> {
  __device__ __forceinline__ static float at(const float* p) { return *p; }
};
template <> struct Stored<uint16_t> {   // BF16 bits -> FP32
  __device__ __forceinline__ static float at(const uint16_t* p) { return __uint_as_float((uint32_t)*p << 16); }
};

// Two adjacent stored values (the first at an even index of an aligned row) in one load.
template <typename TS> struct StoredPair;
template <> struct StoredPair<float> {
  __device__ __forceinline__ static void at(const float* p, float& lo, float& hi) {
    const float2 v = *reinterpret_cast<const float2*>(p);
    lo = v.x;
    hi = v.y;
  }
};
template <> struct StoredPair<uint16_t> {
  __device__ __forceinline__ static void at(const uint16_t* p, float& lo, float& hi) {
    const uint32_t v = *reinterpret_cast<const uint32_t*>(p);
    lo = __uint_as_float(v << 16);
    hi = __uint_as_float(v & 0xffff0000u);
  }
};

// FIT: every term has a target (spline_fit_terms_cells); the targets of a batch are loaded before
// its products, so their latency hides behind the matrix-core work
// LT: some term reads the separate Laplacian table (else its operands take no registers)
// TSET: a term set fixed at compile time (the value alone, the value and Laplacian, all five in
// order, each with its diagonal forms; only without the Laplacian table), else TSET_ANY (each term's
// kind read at run time)
template <typename TS, typename A, int OT, int NT, bool FIT, bool LT, int TSET>
__global__ __launch_bounds__(64)
__attribute__((amdgpu_waves_per_eu(sizeof(A) == 4 && (FIT || (OT == 2 && NT == 5 && !LT)) ? 3 : 1)))
void k_fwd_cells(FwdArgs a) {
  static_assert(TSET == TSET_ANY || (!LT && NT == (TSET == TSET_ALL || TSET == TSET_ALLD ? 5 : 2)),
                "a fixed term set reads the main table, with its own count");
  using M = Mfma<A>;
  using Acc = typename M::acc;
  constexpr int BW = 16 * OT;
  // two tiles: tile ot holds the orbitals ob + 2 col + ot, so each lane's two orbitals are adjacent:
  // their coefficients come in one load and, where the output allows it, their results leave in
  // one 8-byte store (a store instruction then covers 128 contiguous bytes).  Otherwise tile ot
  // holds ob + 16 ot + col.  Not for the FP32 fit terms: their targets load as single values, and
  // with interleaved tiles each such load covers every other word of 128 bytes (0.78 -> 0.82 ms).
  constexpr bool PAIR = OT == 2 && (!FIT || sizeof(TS) == 2);
  bool pst[NT];                                      // term c's outputs take 8-byte stores
#pragma unroll
  for (int c = 0; c < NT; ++c)
    pst[c] = PAIR && c < a.n_terms && ((uintptr_t)a.out[c] & 7) == 0 && (a.out_stride[c] & 1) == 0;
  constexpr int WS = 37;                             // weight row stride in LDS (odd: no bank conflicts)
  __shared__ int s_p[32];
  __shared__ A s_w[32 * WS];                         // per point: x, y, z  x  (w[4], w'[4], w''[4])
  const int lane = (int)threadIdx.x;
  const int grp = lane >> 4;
  const int col = lane & 15;
  // every run before the non-finite points (at most one per occupied cell)
  const int n_runs = (int)min((int64_t)min(max(*a.finite_runs, 0), a.n_pts), a.n_cells);
  const int64_t n_work = (int64_t)n_runs * a.n_groups;
  const int nt = a.n_terms;
  const SortedPoint<A>* pts = static_cast<const SortedPoint<A>*>(a.pts);
  const TS* tab = static_cast<const TS*>(a.table);
  A jm[9], mt[6];
#pragma unroll
  for (int i = 0; i < 9; ++i) jm[i] = (A)a.g.jac[i];
#pragma unroll
  for (int i = 0; i < 6; ++i) mt[i] = (A)a.g.metric[i];

  for (int64_t w = blockIdx.x; w < n_work; w += gridDim.x) {
    const int r = (int)(w / a.n_groups);
    const int ob = (int)(w % a.n_groups) * BW;
    const int64_t cell = a.uniq[r] % a.n_cells;
    const int start = a.offsets[r];
    const int cnt = a.counts[r];
    double sq = 0.0;                                     // this lane's share of the fit terms' sum
    if (cell < 0 || start < 0 || cnt < 0 || start > a.n_pts - cnt) {
      if (FIT && lane == 0) a.partial[w] = 0.0;
      continue;
    }
    const int iz0 = (int)(cell % a.g.n[2]);
    const int iy0 = (int)((cell / a.g.n[2]) % a.g.n[1]);
    const int ix0 = (int)(cell / ((int64_t)a.g.n[2] * a.g.n[1]));
    int ix[4], iy[4], iz[4];
    wrap4(ix0, a.g.n[0], ix);
    wrap4(iy0, a.g.n[1], iy);
    wrap4(iz0, a.g.n[2], iz);
    int orb[OT];                                         // this lane's orbital in tile ot
    bool ocol[OT];
#pragma unroll
    for (int ot = 0; ot < OT; ++ot) {
      orb[ot] = PAIR ? ob + 2 * col + ot : ob + 16 * ot + col;
      ocol[ot] = orb[ot] < a.n_orb;
    }
    // the cell's block as B operands, of the orbital table and (when used) the Laplacian table
    A b0[16][OT], b1[LT ? 16 : 1][OT];
#pragma unroll
    for (int ks = 0; ks < 16; ++ks) {
      const int64_t row = (int64_t)ix[ks >> 2] * a.g.s0 + (int64_t)iy[ks & 3] * a.g.s1 + (int64_t)iz[grp] * a.g.o_pad;
      if constexpr (PAIR) {
        // orb[0] is even and o_pad even, so a pair that starts below n_orb ends inside the row
        // (the second value may be zero padding, whose output is never stored)
        if (ocol[0]) {
          StoredPair<TS>::at(tab + row + orb[0], b0[ks][0], b0[ks][1]);
          if constexpr (LT) StoredPair<TS>::at(tab + a.lap_off + row + orb[0], b1[ks][0], b1[ks][1]);
        } else {
          b0[ks][0] = b0[ks][1] = A(0);
          if constexpr (LT) b1[ks][0] = b1[ks][1] = A(0);
        }
      } else {
#pragma unroll
        for (int ot = 0; ot < OT; ++ot) {
          const int64_t at = row + orb[ot];
          b0[ks][ot] = ocol[ot] ? (A)Stored<TS>::at(tab + at) : A(0);
          if constexpr (LT) b1[ks][ot] = ocol[ot] ? (A)Stored<TS>::at(tab + a.lap_off + at) : A(0);
        }
      }
    }
    for (int b0p = 0; b0p < cnt; b0p += 32) {
      const int nb = min(32, cnt - b0p);
      __syncthreads();                                   // the previous batch is written out
      if (lane < nb) {
        const SortedPoint<A> sp = pts[start + b0p + lane];
        s_p[lane] = (unsigned)sp.p < (unsigned)a.n_pts ? sp.p : -1;   // -1: not written
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          A w4[4], d4[4], dd4[4];
          bspline_weights<A>(sp.t[ax], w4, d4, dd4);
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            s_w[lane * WS + 12 * ax + i] = w4[i];
            s_w[lane * WS + 12 * ax + 4 + i] = d4[i];
            s_w[lane * WS + 12 * ax + 8 + i] = dd4[i];
          }
        }
      }
      __syncthreads();
      const int tiles = nb > 16 ? 2 : 1;
      // one tile of 16 points at a time (targets, products, write-out): half the registers of
      // both tiles at once
#pragma unroll
      for (int mt_ = 0; mt_ < 2; ++mt_) {
        if (mt_ >= tiles) break;
        // fit: every lane loads the targets of its outputs without branching (an entry with no
        // output reads element 0 instead and goes unused), so the loads stay countable and one
        // wait after the products covers them
        A tg[FIT ? NT : 1][OT][4];
        if constexpr (FIT) {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int j = mt_ * 16 + M::row(grp, e);
            const int64_t p = j < nb ? s_p[j] : -1;
#pragma unroll
            for (int c = 0; c < NT; ++c) {
              const int cc = c < nt ? c : 0;
              const A* base = static_cast<const A*>(a.target[cc]);
#pragma unroll
              for (int ot = 0; ot < OT; ++ot) {
                const bool ok = c < nt && p >= 0 && ocol[ot];
                tg[c][ot][e] = base[ok ? p * a.out_stride[cc] + orb[ot] : 0];
              }
            }
          }
        }
        Acc acc[NT][OT];
#pragma unroll
        for (int c = 0; c < NT; ++c)
#pragma unroll
          for (int ot = 0; ot < OT; ++ot) acc[c][ot] = Acc{};
        // row (l, m, n) of k-step 4 l + m, lane group n: per point and m each term's weight is
        // Q2 w_x''[l] + Q1 w_x'[l] + Q0 w_x[l], with Q0..Q2 from the y and z weights (as in the adjoint)
        const A* wp = s_w + min(mt_ * 16 + col, nb - 1) * WS;     // points past nb multiply valid weights
        A wx[4], dwx[4], d2wx[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          wx[i] = wp[i];
          dwx[i] = wp[4 + i];
          d2wx[i] = wp[8 + i];
        }
        const A wz = wp[24 + grp], dwz = wp[28 + grp], d2wz = wp[32 + grp];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const A wy = wp[12 + m], dwy = wp[16 + m], d2wy = wp[20 + m];
#pragma unroll
          for (int c = 0; c < NT; ++c) {
            if (c >= nt) break;
            const int kind = TSET == TSET_ANY ? a.kind[c]
                             : (TSET == TSET_V ? TERM_VAL
                                               : (TSET == TSET_VL || TSET == TSET_VLD ? (c == 0 ? TERM_VAL : TERM_LAP) : c));
            A avs[4];
            row_weights<A, TSET>(c, kind, wx, dwx, d2wx, wy, dwy, d2wy, wz, dwz, d2wz, jm, mt, avs);
            const bool lt = a.src[c] != 0;
#pragma unroll
            for (int l = 0; l < 4; ++l) {
              const A av = avs[l];
#pragma unroll
              for (int ot = 0; ot < OT; ++ot)
                acc[c][ot] = M::step(av, (LT && lt) ? b1[LT ? 4 * l + m : 0][ot] : b0[4 * l + m][ot], acc[c][ot]);
            }
          }
        }
        // vmcnt(0): the targets have arrived (the products took far longer than the loads)
        if constexpr (FIT) __builtin_amdgcn_s_waitcnt(0x0f70);
        // out[point][o]: element e of lane (grp, col) is point row(grp, e) of the tile, orbital col
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int j = mt_ * 16 + M::row(grp, e);
          if (j >= nb || s_p[j] < 0) continue;
          const int64_t p = s_p[j];
#pragma unroll
          for (int c = 0; c < NT; ++c) {
            if (c >= nt) break;
            A* out = static_cast<A*>(a.out[c]) + p * a.out_stride[c];
            A y[OT];
            if constexpr (FIT) {
              const A two_w = (A)(2.0 * a.w[c]);
#pragma unroll
              for (int ot = 0; ot < OT; ++ot) {
                const A res = acc[c][ot][e] - tg[c][ot][e];
                y[ot] = two_w * res;
                if (ocol[ot]) sq = fma(a.w[c] * (double)res, (double)res, sq);
              }
            } else {
#pragma unroll
              for (int ot = 0; ot < OT; ++ot) y[ot] = acc[c][ot][e];
            }
            if constexpr (PAIR) {
              if (pst[c] && ocol[1]) {
                *reinterpret_cast<float2*>(out + orb[0]) = make_float2(y[0], y[1]);
                continue;
              }
            }
#pragma unroll
            for (int ot = 0; ot < OT; ++ot)
              if (ocol[ot]) out[orb[ot]] = y[ot];
          }
        }
      }
    }
    if constexpr (FIT) {
      // the wave's sum in a fixed butterfly order, one slot per work item
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) sq += __shfl_xor(sq, off);
      if (lane == 0) a.partial[w] = sq;
    }
  }
}

// ---------------------------------------------------------------------------------------------
// The fit's data-term gradient in one pass (spline_fit_gradient_cells): FP32 table, value and
// derivative-Laplacian terms, dense points.  Per brick of 2 x 2 x 2 cells and batch of a cell's
// points: the forward values of both terms on the matrix cores from the cell's block (as
// k_fwd_cells), the residuals against the targets, the loss terms and the upstream gradient
// 2 w (y - t) (as the fit terms), and at once the adjoint products of that gradient into the
// brick's region (as k_bwd_bricks).  The upstream gradient stays in registers: the forward's output
// layout (lane group k holds points 4 k .. 4 k + 3 of a tile) becomes the adjoint's operand layout
// (k-step q: lane group k holds point 4 q + k) by a 4 x 4 transpose across lane groups, two rounds
// of 32- and 16-lane swaps.  Every sum is formed as in those two kernels and in the same order, so
// the loss partials and the region sums are the same bits as spline_fit_terms_cells followed by
// the deterministic adjoint (with a diagonal metric, the same numbers: see DIAG below).
struct FitArgs {
  Geom g;
  const float* table;
  int32_t table_bytes;         // under 2 GiB (buffer loads with 32-bit offsets)
  const float* target[2];      // t_v, t_lap: [n_pts][n_orb], the caller's point order
  int32_t target_bytes[2];     // each under 2 GiB
  double w[2];                 // the terms' weights
  const int32_t* cell_range;   // [n_cells][3]: first sorted point, count (0: empty), run index
  const void* pts;             // SortedPoint<float> records in sorted order
  void* blocks;                // [n_bricks][125][o_pad] regions
  double* partial;             // [runs][n_groups] loss partial sums
  int32_t n_pts, n_orb, o_pad, n_groups, n_runs;
};

// 4 x 4 transpose across the lane groups of a wave: register e of lane group k becomes register k of
// lane group e (lane order within a group kept).
__device__ __forceinline__ void transpose_groups(float (&x)[4]) {
  auto a02 = __builtin_amdgcn_permlane32_swap(__float_as_uint(x[0]), __float_as_uint(x[2]), false, false);
  auto a13 = __builtin_amdgcn_permlane32_swap(__float_as_uint(x[1]), __float_as_uint(x[3]), false, false);
  auto b01 = __builtin_amdgcn_permlane16_swap(a02[0], a13[0], false, false);
  auto b23 = __builtin_amdgcn_permlane16_swap(a02[1], a13[1], false, false);
  x[0] = __uint_as_float(b01[0]);
  x[1] = __uint_as_float(b01[1]);
  x[2] = __uint_as_float(b23[0]);
  x[3] = __uint_as_float(b23[1]);
}

// DIAG: the metric M = J J^T is diagonal (orthogonal lattice vectors, as in the cubic cells), so the
// Laplacian's mixed terms vanish: Q1 = 0 and Q0 loses its 2 M12 term.  Those products are exact
// zeros in the general form, so every row weight is the same number either way (an exact zero may
// differ in sign); the diagonal form skips them, about 13% of the kernel's vector instructions.
template <bool DIAG>
__global__ __launch_bounds__(64 * BRICK_WAVES) __attribute__((amdgpu_waves_per_eu(2))) void k_fit_bricks(FitArgs a) {
  using A = float;
  using M = Mfma<float>;
  using Acc = M::acc;
  constexpr int OT = 2;                                // orbital tiles of 16 per wave
  constexpr int BW = 16 * OT;
  constexpr int WBW = BRICK_WAVES * BW;
  constexpr uint32_t RSRC = 0x00020000;                // raw buffer resource, range-checked
  __shared__ int s_p[2][CELL_PB];
  __shared__ A s_w[2][CELL_PB][36];
  __shared__ int s_rng[24];
  __shared__ A s_reg[BRICK_ROWS * WBW];
  const int tid = (int)threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int grp = lane >> 4;
  const int col = lane & 15;
  const int m_ = col >> 2, n_ = col & 3;
  const int nbx = (a.g.n[0] + 1) >> 1, nby = (a.g.n[1] + 1) >> 1, nbz = (a.g.n[2] + 1) >> 1;
  const int64_t n_bricks = (int64_t)nbx * nby * nbz;
  const int n_wg = (a.n_groups + BRICK_WAVES - 1) / BRICK_WAVES;
  const int64_t n_work = n_bricks * n_wg;
  const SortedPoint<A>* pts = static_cast<const SortedPoint<A>*>(a.pts);
  A jm[9], mt[6];
#pragma unroll
  for (int i = 0; i < 9; ++i) jm[i] = (A)a.g.jac[i];
#pragma unroll
  for (int i = 0; i < 6; ++i) mt[i] = (A)a.g.metric[i];
  const A two_w[2] = {(A)(2.0 * a.w[0]), (A)(2.0 * a.w[1])};
  const __amdgpu_buffer_rsrc_t rs_tab =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(a.table), (short)0, a.table_bytes, RSRC);
  const __amdgpu_buffer_rsrc_t rs_t0 =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(a.target[0]), (short)0, a.target_bytes[0], RSRC);
  const __amdgpu_buffer_rsrc_t rs_t1 =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(a.target[1]), (short)0, a.target_bytes[1], RSRC);
  const uint32_t row_bytes = (uint32_t)a.n_orb * 4u;  // target row stride

  for (int64_t w = blockIdx.x; w < n_work; w += gridDim.x) {
    const int64_t brick = w / n_wg;
    const int obw = (int)(w % n_wg) * WBW;
    const int ob = obw + wave * BW;                    // first orbital of this wave
    const int group = ob / BW;                         // the wave's group of 32 orbitals (loss slot)
    const int bz = (int)(brick % nbz);
    const int by = (int)((brick / nbz) % nby);
    const int bx = (int)(brick / ((int64_t)nbz * nby));
    // the lane's orbital in tile ot: ob + 16 ot + col (as the FP32 fit terms); an orbital past
    // n_orb sets bit 31 of its offsets, which reads 0
    uint32_t col_off[OT], col_flag[OT], col_tgt[OT];
    bool ocol[OT];
#pragma unroll
    for (int ot = 0; ot < OT; ++ot) {
      ocol[ot] = ob + 16 * ot + col < a.n_orb;
      col_off[ot] = ocol[ot] ? (uint32_t)(ob + 16 * ot + col) * 4u : 0u;
      col_flag[ot] = ocol[ot] ? 0u : 0x80000000u;
      col_tgt[ot] = ocol[ot] ? col_off[ot] : 0x80000000u;
    }
    __syncthreads();                                   // the previous region is written out
    for (int i = tid; i < BRICK_ROWS * WBW; i += 64 * BRICK_WAVES) s_reg[i] = A(0);
    if (tid < 8) {
      const int X = 2 * bx + (tid >> 2), Y = 2 * by + ((tid >> 1) & 1), Z = 2 * bz + (tid & 1);
      int start = 0, cnt = 0, run = -1;
      if (X < a.g.n[0] && Y < a.g.n[1] && Z < a.g.n[2]) {
        const int64_t cell = ((int64_t)X * a.g.n[1] + Y) * a.g.n[2] + Z;
        start = a.cell_range[3 * cell];
        cnt = a.cell_range[3 * cell + 1];
        run = a.cell_range[3 * cell + 2];
        if (start < 0 || cnt < 0 || start > a.n_pts - cnt) cnt = 0;
      }
      s_rng[tid] = start;
      s_rng[8 + tid] = cnt;
      s_rng[16 + tid] = run;
    }
    __syncthreads();
    const int lane_start = s_rng[lane & 7], lane_count = s_rng[8 + (lane & 7)], lane_run = s_rng[16 + (lane & 7)];
    auto start_of = [&](int c) { return __builtin_amdgcn_readlane(lane_start, c); };
    auto count_of = [&](int c) { return __builtin_amdgcn_readlane(lane_count, c); };
    auto run_of = [&](int c) { return __builtin_amdgcn_readlane(lane_run, c); };
    auto advance = [&](BrickBatch& b) {
      if (b.c >= 8) return;
      b.b0 += CELL_PB;
      if (b.b0 >= count_of(b.c)) {
        b.b0 = 0;
        ++b.c;
        while (b.c < 8 && count_of(b.c) == 0) ++b.c;
      }
    };
    auto count = [&](const BrickBatch& b) { return b.c < 8 ? min(CELL_PB, count_of(b.c) - b.b0) : 0; };
    // staging, as in k_bwd_bricks: thread 3 j + ax holds point j's coordinate on axis ax
    const int sj = tid / 3, sax = tid - 3 * sj;
    struct Staged {
      A t;
      int p;
    };
    auto load_points = [&](const BrickBatch& b, Staged& sp) {
      const int64_t k = min(max((int64_t)start_of(min(b.c, 7)) + b.b0 + sj, (int64_t)0), (int64_t)a.n_pts - 1);
      const SortedPoint<A>* rec = pts + k;
      sp.t = rec->t[sax];
      sp.p = rec->p;
    };
    // a point's target row as a byte offset (under 2^31 - 4096: each target array is under that);
    // none: bit 31 alone
    auto stage_index = [&](const BrickBatch& b, const Staged& sp, int* sp_out) {
      if (sax == 0 && sj < count(b))
        sp_out[sj] = (unsigned)sp.p < (unsigned)a.n_pts ? (int)((uint32_t)sp.p * row_bytes) : (int)0x80000000u;
    };
    auto stage_weights = [&](const BrickBatch& b, const Staged& sp, A (*sw)[36]) {
      if (sj < count(b)) {
        A w4[4], d4[4], dd4[4];
        bspline_weights<A>(sp.t, w4, d4, dd4);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          sw[sj][12 * sax + i] = w4[i];
          sw[sj][12 * sax + 4 + i] = d4[i];
          sw[sj][12 * sax + 8 + i] = dd4[i];
        }
      }
    };
    // the cell's block as the forward's B operands: k-step 4 l + m, lane group n holds row (l, m, n)
    auto load_block = [&](int c, A (&blk)[16][OT]) {
      const int X = 2 * bx + (c >> 2), Y = 2 * by + ((c >> 1) & 1), Z = 2 * bz + (c & 1);
      int ix[4], iy[4], iz[4];
      wrap4(min(X, a.g.n[0] - 1), a.g.n[0], ix);
      wrap4(min(Y, a.g.n[1] - 1), a.g.n[1], iy);
      wrap4(min(Z, a.g.n[2] - 1), a.g.n[2], iz);
      // the lane's part of the offset (third axis, orbital) in the vector offset, the part shared by
      // the wave (first two axes) in the scalar offset; an orbital past n_orb sets bit 31 of the
      // vector offset, out of range with or without the scalar part
      uint32_t voff[OT];
#pragma unroll
      for (int ot = 0; ot < OT; ++ot) voff[ot] = ((uint32_t)iz[grp] * (uint32_t)a.g.o_pad * 4u + col_off[ot]) | col_flag[ot];
#pragma unroll
      for (int ks = 0; ks < 16; ++ks) {
        const int soff = (int)((uint32_t)((int64_t)ix[ks >> 2] * a.g.s0 + (int64_t)iy[ks & 3] * a.g.s1) * 4u);
#pragma unroll
        for (int ot = 0; ot < OT; ++ot)
          blk[ks][ot] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs_tab, voff[ot], soff, 0));
      }
    };
    // the targets of a batch, in the forward's output layout: tile mt, lane group k, element e is
    // point 16 mt + 4 k + e; bit 4 mt + e of `valid` marks a point that is written (as the fit terms)
    auto load_targets = [&](int nb, const int* sp_in, A (&tg)[2][2][OT][4], uint32_t& valid) {
      valid = 0;
#pragma unroll
      for (int mt_ = 0; mt_ < 2; ++mt_)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int j = mt_ * 16 + M::row(grp, e);            // under CELL_PB
          // past the batch: bit 31 set over a stale entry (no select of a loaded value, which the
          // compiler would make a branch of)
          const int pj = sp_in[j] | (int)((uint32_t)(j >= nb) << 31);
          const bool live = pj >= 0;
          valid |= live ? 1u << (4 * mt_ + e) : 0u;
#pragma unroll
          for (int ot = 0; ot < OT; ++ot) {
            // one add: a live point and orbital give the value's offset; a dead orbital (bit 31 in
            // col_tgt) on a live row stays past the array and reads 0; a dead point may wrap into the
            // array, and its value is never used (`valid`)
            const uint32_t off = (uint32_t)pj + col_tgt[ot];
            tg[mt_][0][ot][e] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs_t0, off, 0, 0));
            tg[mt_][1][ot][e] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs_t1, off, 0, 0));
          }
        }
    };
    Acc acc[4][OT];                                    // the cell's block gradient (adjoint)
    double sq = 0.0;                                   // this lane's share of the cell's loss terms
    A blk[16][OT];                                     // the current cell's block
    // forward, residuals and adjoint of one tile of 16 points of the current batch; next_cell >= 0:
    // this is the cell's last tile, and once its forward products are issued, the block registers
    // take the next cell's block (its loads overlap the residuals and the adjoint)
    auto tile = [&](int nb, int mt_, const A (*sw)[36], const A (&tg)[2][2][OT][4], uint32_t valid, int next_cell) {
      Acc accf[2][OT];
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int ot = 0; ot < OT; ++ot) accf[c][ot] = Acc{};
      {
        // forward (as k_fwd_cells): lane col is point 16 mt + col, k-steps run over the block rows
        const A* wp = sw[min(mt_ * 16 + col, nb - 1)];
        A wx[4], dwx[4], d2wx[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          wx[i] = wp[i];
          dwx[i] = wp[4 + i];
          d2wx[i] = wp[8 + i];
        }
        const A wz = wp[24 + grp], dwz = wp[28 + grp], d2wz = wp[32 + grp];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const A wy = wp[12 + m], dwy = wp[16 + m], d2wy = wp[20 + m];
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            A q0, q1, q2;
            if (DIAG && c == 1) lap_factors_diag<A>(wy, d2wy, wz, d2wz, mt, q0, q1, q2);
            else term_factors<A>(c == 0 ? TERM_VAL : TERM_LAP, wy, dwy, d2wy, wz, dwz, d2wz, jm, mt, q0, q1, q2);
#pragma unroll
            for (int l = 0; l < 4; ++l) {
              // the value term: the vanishing Q1, Q2 products change no bit of q0 w_x (finite,
              // non-negative weights)
              const A av = c == 0 ? q0 * wx[l] : (DIAG ? fmaa(q2, d2wx[l], q0 * wx[l]) : fmaa(q2, d2wx[l], fmaa(q1, dwx[l], q0 * wx[l])));
#pragma unroll
              for (int ot = 0; ot < OT; ++ot) accf[c][ot] = M::step(av, blk[4 * l + m][ot], accf[c][ot]);
            }
          }
        }
      }
      if (next_cell >= 0) load_block(next_cell, blk);
      // residuals, loss terms and upstream gradient (as the fit terms); zero for points not written
      A gd[2][OT][4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const bool ok = (valid >> (4 * mt_ + e)) & 1u;
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
          for (int ot = 0; ot < OT; ++ot) {
            // an entry not written adds w 0 0 = +-0 (w finite) to a sum that starts at +0 and so is
            // never -0: the same bits as skipping it, with no branch (the compiler branches on a
            // select of a loaded value)
            const bool use = ok && ocol[ot];
            const A res = accf[c][ot][e] - tg[mt_][c][ot][e];
            const double rd = (double)(use ? res : A(0));
            sq = fma(a.w[c] * rd, rd, sq);
            gd[c][ot][e] = use ? two_w[c] * res : A(0);
          }
      }
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int ot = 0; ot < OT; ++ot) transpose_groups(gd[c][ot]);
      // adjoint (as k_bwd_bricks): k-step 4 mt + q takes points 16 mt + 4 q + (lane group)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int qs = mt_ * 16 + 4 * q;
        if (qs >= nb) break;
        const A* wp = sw[min(qs + grp, nb - 1)];
        A wx[4], dwx[4], d2wx[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          wx[i] = wp[i];
          dwx[i] = wp[4 + i];
          d2wx[i] = wp[8 + i];
        }
        const A wy = wp[12 + m_], dwy = wp[16 + m_], d2wy = wp[20 + m_];
        const A wz = wp[24 + n_], dwz = wp[28 + n_], d2wz = wp[32 + n_];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          A q0, q1, q2;
          if (DIAG && c == 1) lap_factors_diag<A>(wy, d2wy, wz, d2wz, mt, q0, q1, q2);
          else term_factors<A>(c == 0 ? TERM_VAL : TERM_LAP, wy, dwy, d2wy, wz, dwz, d2wz, jm, mt, q0, q1, q2);
#pragma unroll
          for (int rt = 0; rt < 4; ++rt) {
            const A av = c == 0 ? q0 * wx[rt] : (DIAG ? fmaa(q2, d2wx[rt], q0 * wx[rt]) : fmaa(q2, d2wx[rt], fmaa(q1, dwx[rt], q0 * wx[rt])));
#pragma unroll
            for (int ot = 0; ot < OT; ++ot) acc[rt][ot] = M::step(av, gd[c][ot][q], acc[rt][ot]);
          }
        }
      }
    };
    auto add_block = [&](int c) {
      A* corner = s_reg + (((c >> 2) * 5 + ((c >> 1) & 1)) * 5 + (c & 1)) * WBW + wave * BW;
#pragma unroll
      for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int i = M::row(grp, e);
          A* rp = corner + ((rt * 5 + (i >> 2)) * 5 + (i & 3)) * WBW;
#pragma unroll
          for (int ot = 0; ot < OT; ++ot) rp[16 * ot + col] += acc[rt][ot][e];
        }
    };

    BrickBatch b0{0, 0};
    while (b0.c < 8 && count_of(b0.c) == 0) ++b0.c;
    BrickBatch b1 = b0;
    advance(b1);
    BrickBatch b2 = b1;
    advance(b2);
    BrickBatch b3 = b2;
    advance(b3);
    Staged sp0, sp_next, sp_after;
    load_points(b0, sp0);
    load_points(b1, sp_next);
    load_points(b2, sp_after);
    if (b0.c < 8) load_block(b0.c, blk);
    if (tid < 3 * CELL_PB) {
      stage_index(b0, sp0, s_p[0]);
      stage_weights(b0, sp0, s_w[0]);
      stage_index(b1, sp_next, s_p[1]);
    }
    __syncthreads();
    A tgq[2][2][2][OT][4];
    uint32_t vq[2];
    load_targets(count(b0), s_p[0], tgq[0], vq[0]);
    __syncthreads();                                   // every wave has read b0's indices before the first
                                                       // step stages b2's over them
    auto step = [&](int buf, A (&tg_cur)[2][2][OT][4], uint32_t& v_cur, A (&tg_nxt)[2][2][OT][4], uint32_t& v_nxt) {
      const int nb = count(b0);
      load_targets(count(b1), s_p[buf ^ 1], tg_nxt, v_nxt);
      const bool last = b0.b0 + CELL_PB >= count_of(b0.c);     // b0 ends its cell
      const int next_cell = last && b1.c < 8 ? b1.c : -1;
      if (tid < 3 * CELL_PB) {
        stage_weights(b1, sp_next, s_w[buf ^ 1]);
        stage_index(b2, sp_after, s_p[buf]);
      }
      sp_next = sp_after;
      load_points(b3, sp_after);
      if (b0.b0 == 0) {
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
#pragma unroll
          for (int ot = 0; ot < OT; ++ot) acc[rt][ot] = Acc{};
        sq = 0.0;
      }
      tile(nb, 0, s_w[buf], tg_cur, v_cur, nb > 16 ? -1 : next_cell);
      if (nb > 16) tile(nb, 1, s_w[buf], tg_cur, v_cur, next_cell);
      if (last) {
        add_block(b0.c);
        // the cell's loss partial: the wave's sum in a fixed butterfly order (as the fit terms)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) sq += __shfl_xor(sq, off);
        const int run = run_of(b0.c);
        if (lane == 0 && group < a.n_groups && run >= 0 && run < a.n_runs) a.partial[(int64_t)run * a.n_groups + group] = sq;
      }
      __syncthreads();
      b0 = b1;
      b1 = b2;
      b2 = b3;
      advance(b3);
    };
    while (b0.c < 8) {
      step(0, tgq[0], vq[0], tgq[1], vq[1]);
      if (b0.c >= 8) break;
      step(1, tgq[1], vq[1], tgq[0], vq[0]);
    }
    __syncthreads();
    A* out = static_cast<A*>(a.blocks) + brick * BRICK_ROWS * a.o_pad + obw;
    for (int i = tid; i < BRICK_ROWS * WBW; i += 64 * BRICK_WAVES) {
      const int lrow = i / WBW, c = i % WBW;
      if (obw + c < a.n_orb) out[(int64_t)lrow * a.o_pad + c] = s_reg[i];
    }
  }
}

// loss += the work items' partial sums, in a fixed order, in two steps.  First FIT_SUM_BLOCKS
// workgroups: thread t of workgroup b sums the partials b T + t + k (FIT_SUM_BLOCKS T), then a fixed
// tree in LDS gives block sum b.  Then one workgroup adds the block sums in a fixed tree to *loss,
// or NaN when a point is not finite (its terms are NaN, as the misfit of its NaN outputs would be).
__device__ __forceinline__ double block_tree_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int h = FIT_SUM_THREADS / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  return red[0];
}

__global__ __launch_bounds__(FIT_SUM_THREADS) void k_fit_blocks(const int32_t* finite_runs, int32_t n_pts,
                                                                int64_t n_cells, int32_t n_groups,
                                                                const double* partial, double* block_sum) {
  __shared__ double red[FIT_SUM_THREADS];
  const int64_t n_runs = min((int64_t)min(max(*finite_runs, 0), n_pts), n_cells);
  const int64_t n_work = n_runs * n_groups;
  constexpr int64_t S = (int64_t)FIT_SUM_BLOCKS * FIT_SUM_THREADS;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  int64_t i = (int64_t)blockIdx.x * FIT_SUM_THREADS + threadIdx.x;
  for (; i + 3 * S < n_work; i += 4 * S)
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[u] += partial[i + u * S];
#pragma unroll
  for (int u = 0; u < 4; ++u)
    if (i + u * S < n_work) acc[u] += partial[i + u * S];
  const double s = block_tree_sum((acc[0] + acc[1]) + (acc[2] + acc[3]), red);
  if (threadIdx.x == 0) block_sum[blockIdx.x] = s;
}

__global__ __launch_bounds__(FIT_SUM_THREADS) void k_fit_total(const double* block_sum, const int64_t* keys,
                                                               int32_t n_pts, int64_t sentinel, double* loss) {
  __shared__ double red[FIT_SUM_THREADS];
  const double s = block_tree_sum(threadIdx.x < FIT_SUM_BLOCKS ? block_sum[threadIdx.x] : 0.0, red);
  if (threadIdx.x == 0) *loss += keys[n_pts - 1] == sentinel ? (double)__builtin_nan("") : s;
}

// Non-finite points (sorted last under the sentinel key) get NaN in every requested output.
template <typename A>
__global__ __launch_bounds__(256) void k_fwd_nan(const int64_t* keys, const int32_t* perm, int32_t n, int64_t sentinel,
                                                 FwdArgs a) {
  const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i >= n || keys[i] != sentinel) return;
  const int64_t p = perm[i];
  if (p < 0 || p >= n) return;
  const A nan = __builtin_nan("");
  for (int c = 0; c < a.n_terms; ++c) {
    A* out = static_cast<A*>(a.out[c]) + p * a.out_stride[c];
    for (int o = 0; o < a.n_orb; ++o) out[o] = nan;
  }
}

typedef void (*FwdKernel)(FwdArgs);

// FP32 with at most two terms: two orbital tiles per wave; otherwise one (accumulator registers)
// (the fit terms come in at most two: values and Laplacians)
template <typename TS, typename A, bool LT, int TSET>
static FwdKernel pick_fwd_set(int nt, bool fit) {
  constexpr int OT2 = sizeof(A) == 4 ? 2 : 1;   // orbital tiles of the at-most-two-term forms
  if constexpr (TSET == TSET_ALL || TSET == TSET_ALLD) {
    return k_fwd_cells<TS, A, OT2, 5, false, LT, TSET>;
  } else if constexpr (TSET != TSET_ANY) {
    return fit ? k_fwd_cells<TS, A, OT2, 2, true, LT, TSET> : k_fwd_cells<TS, A, OT2, 2, false, LT, TSET>;
  } else {
    if (fit) return k_fwd_cells<TS, A, OT2, 2, true, LT, TSET_ANY>;
    if constexpr (sizeof(A) == 4) {
      if (nt <= 2) return k_fwd_cells<TS, A, 2, 2, false, LT, TSET_ANY>;
      if constexpr (!LT) return k_fwd_cells<TS, A, 2, 5, false, LT, TSET_ANY>;
    }
    return nt <= 2 ? k_fwd_cells<TS, A, 1, 2, false, LT, TSET_ANY> : k_fwd_cells<TS, A, 1, 5, false, LT, TSET_ANY>;
  }
}

// tset: a fixed term set (only without the Laplacian table), else TSET_ANY
template <typename TS, typename A>
static FwdKernel pick_fwd(int nt, bool fit, bool lt, int tset) {
  if (lt) return pick_fwd_set<TS, A, true, TSET_ANY>(nt, fit);
  switch (tset) {
    case TSET_V: return pick_fwd_set<TS, A, false, TSET_V>(nt, fit);
    case TSET_VL: return pick_fwd_set<TS, A, false, TSET_VL>(nt, fit);
    case TSET_VLD: return pick_fwd_set<TS, A, false, TSET_VLD>(nt, fit);
    case TSET_ALL: return pick_fwd_set<TS, A, false, TSET_ALL>(nt, fit);
    case TSET_ALLD: return pick_fwd_set<TS, A, false, TSET_ALLD>(nt, fit);
    default: return pick_fwd_set<TS, A, false, TSET_ANY>(nt, fit);
  }
}

static int fwd_tiles(int dtype, int nt, bool lt) { return dtype != SPL_F64 && (nt <= 2 || !lt) ? 2 : 1; }

int cells_eval_work_bytes(const spl_desc* d, int64_t n_pts, int64_t* bytes) {
  SortLayout L;
  int rc = sort_layout(d, n_pts, &L, false);
  if (rc) return rc;
  *bytes = (int64_t)L.total;
  return SPL_OK;
}

int launch_eval_cells(const spl_desc* d, const void* table, int64_t n_pts, const double* pos, void* v, void* grad,
                      void* lap, void* work, int64_t work_bytes, bool reuse, hipStream_t stream,
                      const FitTerms* fit) {
  if (n_pts == 0) return SPL_OK;
  SortLayout L;
  int rc = sort_layout(d, n_pts, &L, false);
  if (rc) return rc;
  if (!work || work_bytes < (int64_t)L.total)
    return fail(SPL_EINVAL, "spline_eval_vgl_cells needs a workspace of %lld bytes", (long long)L.total);
  CellSort cs;
  if ((rc = cell_sort(d, n_pts, pos, work, L, reuse, stream, &cs))) return rc;
  FwdArgs a;
  memset(&a, 0, sizeof(a));
  a.g = make_geom(d);
  a.table = table;
  a.lap_off = d->has_lap ? d->table_elems : 0;
  const int64_t no = d->n_orb;
  const size_t os = d->dtype == SPL_F64 ? 8 : 4;
  int nt = 0;
  auto term = [&](void* out, int64_t stride, int kind, int src, const void* target = nullptr, double w = 0.0) {
    a.out[nt] = out;
    a.out_stride[nt] = stride;
    a.kind[nt] = kind;
    a.src[nt] = src;
    a.target[nt] = target;
    a.w[nt] = w;
    if (src == 1) a.use_lap_table = 1;
    ++nt;
  };
  if (fit) {
    // fit terms: v and lap receive the upstream gradients of the misfit of values and Laplacians
    if (v) term(v, no, TERM_VAL, 0, fit->t_v, fit->w_v);
    if (lap) {
      if (d->has_lap) term(lap, no, TERM_VAL, 1, fit->t_lap, fit->w_lap);
      else term(lap, no, TERM_LAP, 0, fit->t_lap, fit->w_lap);
    }
    v = grad = nullptr;
    lap = nullptr;
    a.partial = reinterpret_cast<double*>(static_cast<char*>(work) + L.partials);
  }
  if (v) term(v, no, TERM_VAL, 0);
  if (grad) {
    char* gb = static_cast<char*>(grad);
    term(gb, 3 * no, TERM_GX, 0);
    term(gb + no * os, 3 * no, TERM_GY, 0);
    term(gb + 2 * no * os, 3 * no, TERM_GZ, 0);
  }
  if (lap) {
    if (d->has_lap) term(lap, no, TERM_VAL, 1);
    else term(lap, no, TERM_LAP, 0);
  }
  a.n_terms = nt;
  a.uniq = cs.uniq;
  a.counts = cs.counts;
  a.offsets = cs.offsets;
  a.pts = cs.pts;
  a.finite_runs = cs.finite_runs;
  a.n_cells = L.n_cells;
  a.n_pts = (int32_t)n_pts;
  a.n_orb = d->n_orb;
  const int ot = fwd_tiles(d->dtype, nt, a.use_lap_table != 0);
  a.n_groups = (d->n_orb + 16 * ot - 1) / (16 * ot);
  FwdKernel k;
  const bool lt = a.use_lap_table != 0;
  // a term set the kernel fixes at compile time, with its diagonal forms where they apply
  const DiagForms df = diag_forms(d);
  bool all = nt == 5;
  for (int c = 0; c < nt; ++c) all = all && a.kind[c] == TERM_VAL + c;
  int tset = TSET_ANY;
  if (nt == 2 && a.kind[0] == TERM_VAL && a.kind[1] == TERM_LAP) tset = df.diag ? TSET_VLD : TSET_VL;
  else if (all && !fit) tset = df.diag_jac ? TSET_ALLD : TSET_ALL;
  else if (nt == 1 && a.kind[0] == TERM_VAL && !fit) tset = TSET_V;
  if (d->dtype == SPL_F64) k = pick_fwd<double, double>(nt, fit != nullptr, lt, tset);
  else if (d->dtype == SPL_F32) k = pick_fwd<float, float>(nt, fit != nullptr, lt, tset);
  else k = pick_fwd<uint16_t, float>(nt, fit != nullptr, lt, tset);
  const int grid = (int)std::min<int64_t>(std::min<int64_t>(n_pts, L.n_cells) * a.n_groups, 1 << 16);
  hipLaunchKernelGGL(k, dim3(grid), dim3(64), 0, stream, a);
  if ((rc = hip_fail(hipGetLastError(), "cell forward launch"))) return rc;
  const int n = (int)n_pts;
  if (fit) {
    // the block sums follow the work items' partials (at most min(n, cells) runs x 16-orbital tiles)
    double* block_sum = a.partial + std::min<int64_t>(n_pts, L.n_cells) * (int64_t)((d->n_orb + 15) / 16);
    hipLaunchKernelGGL(k_fit_blocks, dim3(FIT_SUM_BLOCKS), dim3(FIT_SUM_THREADS), 0, stream, cs.finite_runs,
                       a.n_pts, L.n_cells, a.n_groups, a.partial, block_sum);
    if ((rc = hip_fail(hipGetLastError(), "fit block sums launch"))) return rc;
    hipLaunchKernelGGL(k_fit_total, dim3(1), dim3(FIT_SUM_THREADS), 0, stream, block_sum, cs.keys, a.n_pts,
                       L.n_cells, fit->loss);
    if ((rc = hip_fail(hipGetLastError(), "fit total launch"))) return rc;
  }
  if (d->dtype == SPL_F64)
    hipLaunchKernelGGL(k_fwd_nan<double>, dim3((n + 255) / 256), dim3(256), 0, stream, cs.keys, cs.perm, n,
                       L.n_cells, a);
  else
    hipLaunchKernelGGL(k_fwd_nan<float>, dim3((n + 255) / 256), dim3(256), 0, stream, cs.keys, cs.perm, n,
                       L.n_cells, a);
  return hip_fail(hipGetLastError(), "non-finite point launch");
}

int fit_gradient_work_bytes(const spl_desc* d, int64_t n_pts, int64_t* bytes) {
  SortLayout L;
  int rc = sort_layout(d, n_pts, &L, true, true);
  if (rc) return rc;
  *bytes = (int64_t)L.total;
  return SPL_OK;
}

// The fit's data terms and their coefficient gradient in one pass (k_fit_bricks), then the per-row
// gather of the brick regions and the loss sums.
int launch_fit_gradient(const spl_desc* d, const void* table, int64_t n_pts, const double* pos, const void* t_v,
                        double w_v, const void* t_lap, double w_lap, void* gtable, double* loss, void* work,
                        int64_t work_bytes, bool reuse, hipStream_t stream) {
  if (n_pts == 0) return SPL_OK;
  if (d->dtype != SPL_F32 || d->has_lap)
    return fail(SPL_EUNSUPPORTED, "the one-pass fit gradient covers FP32 tables with the Laplacian from derivatives");
  const int64_t tgt = n_pts * (int64_t)d->n_orb * 4;
  if (d->table_bytes >= ((int64_t)1 << 31) - 4096 || tgt >= ((int64_t)1 << 31) - 4096)
    return fail(SPL_EUNSUPPORTED, "the one-pass fit gradient needs the table and each target array under 2 GiB");
  SortLayout L;
  int rc = sort_layout(d, n_pts, &L, true, true);
  if (rc) return rc;
  if (!L.dense)
    return fail(SPL_EUNSUPPORTED, "the one-pass fit gradient needs at least 2.5 points per cell (%lld points, %lld cells)",
                (long long)n_pts, (long long)L.n_cells);
  if (!work || work_bytes < (int64_t)L.total)
    return fail(SPL_EINVAL, "spline_fit_gradient_cells needs a workspace of %lld bytes", (long long)L.total);
  CellSort cs;
  if ((rc = cell_sort(d, n_pts, pos, work, L, reuse, stream, &cs))) return rc;
  char* W = cs.base;
  int32_t* cell_range = reinterpret_cast<int32_t*>(W + L.cell_range);
  const int max_runs = (int)std::min<int64_t>(n_pts, L.n_cells);
  if (!reuse) {
    // the cells' point ranges, part of this function's sort: a reused sort comes from an earlier
    // call of this function, which left them in the workspace
    hipLaunchKernelGGL(k_bwd_fill_i32, dim3((unsigned)((3 * L.n_cells + 255) / 256)), dim3(256), 0, stream,
                       cell_range, 3 * L.n_cells, 0);
    if ((rc = hip_fail(hipGetLastError(), "cell range clear launch"))) return rc;
    hipLaunchKernelGGL(k_cell_ranges, dim3((unsigned)((max_runs + 255) / 256)), dim3(256), 0, stream, cs.uniq,
                       cs.counts, cs.offsets, cs.finite_runs, L.n_cells, (int32_t)n_pts, cell_range);
    if ((rc = hip_fail(hipGetLastError(), "cell range launch"))) return rc;
  }
  FitArgs a;
  memset(&a, 0, sizeof(a));
  a.g = make_geom(d);
  a.table = static_cast<const float*>(table);
  a.table_bytes = (int32_t)d->table_bytes;
  a.target[0] = static_cast<const float*>(t_v);
  a.target[1] = static_cast<const float*>(t_lap);
  a.target_bytes[0] = a.target_bytes[1] = (int32_t)tgt;
  a.w[0] = w_v;
  a.w[1] = w_lap;
  a.cell_range = cell_range;
  a.pts = cs.pts;
  a.blocks = W + L.blocks;
  a.partial = reinterpret_cast<double*>(W + L.partials);
  a.n_pts = (int32_t)n_pts;
  a.n_orb = d->n_orb;
  a.o_pad = d->o_pad;
  a.n_groups = (d->n_orb + 31) / 32;                 // as the FP32 fit terms: 32 orbitals per work item
  a.n_runs = max_runs;
  const int64_t n_bricks = (int64_t)((d->grid[0] + 1) / 2) * ((d->grid[1] + 1) / 2) * ((d->grid[2] + 1) / 2);
  const int64_t n_wg = (a.n_groups + BRICK_WAVES - 1) / BRICK_WAVES;
  hipLaunchKernelGGL(diag_forms(d).diag ? k_fit_bricks<true> : k_fit_bricks<false>, dim3((unsigned)std::min<int64_t>(n_bricks * n_wg, 1 << 16)),
                     dim3(64 * BRICK_WAVES), 0, stream, a);
  if ((rc = hip_fail(hipGetLastError(), "fit gradient launch"))) return rc;
  if ((rc = launch_brick_gather<float>(d, a.g, a.blocks, gtable, stream))) return rc;
  // the loss: the same two fixed-order sums over the same partials as the fit terms
  double* block_sum = a.partial + std::min<int64_t>(n_pts, L.n_cells) * (int64_t)((d->n_orb + 15) / 16);
  hipLaunchKernelGGL(k_fit_blocks, dim3(FIT_SUM_BLOCKS), dim3(FIT_SUM_THREADS), 0, stream, cs.finite_runs,
                     a.n_pts, L.n_cells, a.n_groups, a.partial, block_sum);
  if ((rc = hip_fail(hipGetLastError(), "fit block sums launch"))) return rc;
  hipLaunchKernelGGL(k_fit_total, dim3(1), dim3(FIT_SUM_THREADS), 0, stream, block_sum, cs.keys, a.n_pts,
                     L.n_cells, loss);
  return hip_fail(hipGetLastError(), "fit total launch");
}

}  // namespace pws


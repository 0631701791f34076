// spline_build: interpolating periodic B-spline coefficients (App. A, Interpolating
// B-spline coefficients).
//
// The coefficients solve (B_1 x B_2 x B_3) beta = f where each B_d is the periodic
// tridiagonal matrix with rows (1/6, 4/6, 1/6) and corner elements.  As in the paper,
// the Kronecker system is solved in three stages, one grid axis at a time; each stage
// solves one cyclic system per grid line, lines being independent.
//
// Per line, the cyclic system is solved exactly through the factorization
//   (1/6)(4 I + S + S^-1) = (1 / (6 lam)) (I + lam S)(I + lam S^-1),  lam = 2 - sqrt(3),
// S the cyclic shift.  Each factor is a first-order cyclic recursion: one pass that
// needs the closed-form start value sum_j (-lam)^j d_{-j} / (1 - (-lam)^n), then a
// sweep.  Two sweeps plus two start sums, about 4 FMA per element, no pivoting (|lam| < 1).
//
// Layout: data is viewed as [outer][n][inner] with the solved axis in the middle; the
// third-axis stage has inner = n_col and writes straight into the padded table in the
// storage dtype (one rounding, FP64 -> FP32 -> BF16, round to nearest even).  A
// workgroup stages `tile` consecutive lines in LDS ([n][tile], conflict-free), so each
// element is read from and written to HBM once per stage.
#include <math.h>

#include "common.hpp"
#include "update.hpp"

namespace pws {

struct LineArgs {
  const double* src;
  void* dst;
  int64_t n_lines;
  int64_t inner;
  int32_t n;
  int32_t o_pad;      // table row stride when writing the table
  double lam;         // 2 - sqrt(3)
  double start_inv;   // 1 / (1 - (-lam)^n)
  double scale;       // 6 lam
};

enum { OUT_F64_WORK = 0, OUT_TABLE_F64 = 1, OUT_TABLE_F32 = 2, OUT_TABLE_BF16 = 3 };

template <int OUT>
__global__ __launch_bounds__(256) void k_cyclic_axis(LineArgs a) {
  extern __shared__ double lds[];
  const int tile = blockDim.x;
  const int tid = threadIdx.x;
  const int64_t line = (int64_t)blockIdx.x * tile + tid;
  if (line >= a.n_lines) return;            // no barriers below: each thread owns its column
  const int n = a.n;
  const int64_t outer = line / a.inner;
  const int64_t in = line - outer * a.inner;
  const int64_t base = outer * (int64_t)n * a.inner + in;
  double* x = lds + tid;

  for (int k = 0; k < n; ++k) x[k * tile] = a.src[base + (int64_t)k * a.inner];

  const double lam = a.lam;
  const double nl = -lam;
  // (I + lam S) y = d:  y_k + lam y_{k-1} = d_k (cyclic)
  double acc = x[0];
  double pw = 1.0;
  for (int j = 1; j < n; ++j) {
    pw *= nl;
    acc = fmaa(pw, x[(n - j) * tile], acc);
  }
  double prev = acc * a.start_inv;
  x[0] = prev;
  for (int k = 1; k < n; ++k) {
    prev = fmaa(-lam, prev, x[k * tile]);
    x[k * tile] = prev;
  }
  // (I + lam S^-1) z = y:  z_k + lam z_{k+1} = y_k (cyclic)
  acc = x[(n - 1) * tile];
  pw = 1.0;
  for (int j = 1; j < n; ++j) {
    pw *= nl;
    acc = fmaa(pw, x[(j - 1) * tile], acc);
  }
  double next = acc * a.start_inv;
  x[(n - 1) * tile] = next;
  for (int k = n - 2; k >= 0; --k) {
    next = fmaa(-lam, next, x[k * tile]);
    x[k * tile] = next;
  }

  if constexpr (OUT == OUT_F64_WORK) {
    double* dst = static_cast<double*>(a.dst);
    for (int k = 0; k < n; ++k) dst[base + (int64_t)k * a.inner] = a.scale * x[k * tile];
  } else {
    const int64_t row0 = outer * (int64_t)n;     // table row of (outer, k = 0); inner == n_col
    for (int k = 0; k < n; ++k) {
      const double val = a.scale * x[k * tile];
      const int64_t idx = (row0 + k) * a.o_pad + in;
      if constexpr (OUT == OUT_TABLE_F64) static_cast<double*>(a.dst)[idx] = val;
      else if constexpr (OUT == OUT_TABLE_F32) static_cast<float*>(a.dst)[idx] = (float)val;
      else static_cast<uint16_t*>(a.dst)[idx] = f32_to_bf16_rne((float)val);
    }
  }
}

// Zero the padding columns [n_col, o_pad) of every table row.
template <typename TS>
__global__ __launch_bounds__(256) void k_zero_pad(TS* table, int64_t n_rows, int32_t n_col, int32_t o_pad) {
  const int32_t width = o_pad - n_col;
  const int64_t total = n_rows * width;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / width;
    table[r * o_pad + n_col + (i - r * width)] = TS(0);
  }
}

// Lagrange tables (App. A, Eq. lagrangeinterpolation3): the coefficients are the grid values,
// rounded once into the storage dtype; padding columns are zeroed.  One element of the padded
// table per iteration: vals [rows][n_col] FP64 -> table [rows][o_pad].
template <int OUT>
__global__ __launch_bounds__(256) void k_cast_table(const double* vals, void* table, int64_t n_rows, int32_t n_col,
                                                    int32_t o_pad) {
  const int64_t total = n_rows * o_pad;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / o_pad;
    const int32_t c = (int32_t)(i - r * o_pad);
    const double x = c < n_col ? vals[r * n_col + c] : 0.0;
    if constexpr (OUT == OUT_TABLE_F64) static_cast<double*>(table)[i] = x;
    else if constexpr (OUT == OUT_TABLE_F32) static_cast<float*>(table)[i] = (float)x;
    else static_cast<uint16_t*>(table)[i] = f32_to_bf16_rne((float)x);
  }
}

static int line_tile(int n) {
  int tile = 256;
  while (tile > 8 && (int64_t)tile * n * 8 > 65536) tile >>= 1;
  return tile;
}

static int launch_axis(int out, const double* src, void* dst, int64_t outer, int n, int64_t inner,
                       int o_pad, hipStream_t stream) {
  LineArgs a;
  a.src = src;
  a.dst = dst;
  a.n_lines = outer * inner;
  a.inner = inner;
  a.n = n;
  a.o_pad = o_pad;
  a.lam = 2.0 - sqrt(3.0);
  a.start_inv = 1.0 / (1.0 - pow(-a.lam, (double)n));
  a.scale = 6.0 * a.lam;
  const int tile = line_tile(n);
  const dim3 grid((unsigned)((a.n_lines + tile - 1) / tile));
  const size_t shmem = (size_t)tile * n * sizeof(double);
  switch (out) {
    case OUT_F64_WORK: hipLaunchKernelGGL(k_cyclic_axis<OUT_F64_WORK>, grid, dim3(tile), shmem, stream, a); break;
    case OUT_TABLE_F64: hipLaunchKernelGGL(k_cyclic_axis<OUT_TABLE_F64>, grid, dim3(tile), shmem, stream, a); break;
    case OUT_TABLE_F32: hipLaunchKernelGGL(k_cyclic_axis<OUT_TABLE_F32>, grid, dim3(tile), shmem, stream, a); break;
    default: hipLaunchKernelGGL(k_cyclic_axis<OUT_TABLE_BF16>, grid, dim3(tile), shmem, stream, a); break;
  }
  return hip_fail(hipGetLastError(), "cyclic solve launch");
}

// Build one B-spline table (orbital, gradient component or Laplacian) from FP64 grid values
// [N1][N2][N3][n_col] into `table` (element offset applied).
int build_one(const spl_desc* d, const double* vals, void* table, double* work, hipStream_t stream) {
  const int64_t n1 = d->grid[0], n2 = d->grid[1], n3 = d->grid[2], no = d->n_col;
  int rc;
  // stage 1: first axis, lines over (j, k, o): [1][N1][N2*N3*O], grid values -> work
  if ((rc = launch_axis(OUT_F64_WORK, vals, work, 1, (int)n1, n2 * n3 * no, 0, stream))) return rc;
  // stage 2: second axis, [N1][N2][N3*O], in place
  if ((rc = launch_axis(OUT_F64_WORK, work, work, n1, (int)n2, n3 * no, 0, stream))) return rc;
  // stage 3: third axis, [N1*N2][N3][O], written into the padded table in the storage dtype
  const int out = d->dtype == SPL_F64 ? OUT_TABLE_F64 : d->dtype == SPL_F32 ? OUT_TABLE_F32 : OUT_TABLE_BF16;
  if ((rc = launch_axis(out, work, table, n1 * n2, (int)n3, no, d->o_pad, stream))) return rc;
  if (d->o_pad > d->n_col) {
    const int64_t rows = n1 * n2 * n3;
    const int64_t total = rows * (d->o_pad - d->n_col);
    const dim3 grid((unsigned)((total + 255) / 256 < 65536 ? (total + 255) / 256 : 65536));
    if (d->dtype == SPL_F64)
      hipLaunchKernelGGL(k_zero_pad<double>, grid, dim3(256), 0, stream, (double*)table, rows, d->n_col, d->o_pad);
    else if (d->dtype == SPL_F32)
      hipLaunchKernelGGL(k_zero_pad<float>, grid, dim3(256), 0, stream, (float*)table, rows, d->n_col, d->o_pad);
    else
      hipLaunchKernelGGL(k_zero_pad<uint16_t>, grid, dim3(256), 0, stream, (uint16_t*)table, rows, d->n_col,
                         d->o_pad);
    if ((rc = hip_fail(hipGetLastError(), "zero padding launch"))) return rc;
  }
  return SPL_OK;
}

// pp-spline table (App. A, Piecewise-polynomial-form splines) from B-spline coefficients beta, FP64
// [N1][N2][N3][n_col].  At a knot the cubic B-spline's value weights are (1, 4, 1)/6 and its
// second-derivative weights (1, -2, 1) in grid units, so each of the 8 numbers of a grid point,
// sigma^{kx ky kz} (Eq. pp-splinecoefficients3), filters beta along every axis with one of the two;
// the three filters are applied one axis after the other (z, then y, then x).  Stored at
// [point][q][o_pad], q = 4 (kx - 1) + 2 (ky - 1) + (kz - 1); padding columns are zeroed.
template <int OUT>
__global__ __launch_bounds__(256) void k_pp_sigma(const double* beta, void* table, int32_t n1, int32_t n2,
                                                  int32_t n3, int32_t n_col, int32_t o_pad) {
  const int64_t pts = (int64_t)n1 * n2 * n3;
  const int64_t total = pts * o_pad;
  const double sixth = 1.0 / 6.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = i / o_pad;
    const int c = (int)(i - p * o_pad);
    double sig[8];
    if (c < n_col) {
      const int i3 = (int)(p % n3);
      const int64_t r = p / n3;
      const int i2 = (int)(r % n2);
      const int i1 = (int)(r / n2);
      const int xi[3] = {i1 == 0 ? n1 - 1 : i1 - 1, i1, i1 + 1 == n1 ? 0 : i1 + 1};
      const int yi[3] = {i2 == 0 ? n2 - 1 : i2 - 1, i2, i2 + 1 == n2 ? 0 : i2 + 1};
      const int zi[3] = {i3 == 0 ? n3 - 1 : i3 - 1, i3, i3 + 1 == n3 ? 0 : i3 + 1};
      double zs[2][3][3];   // [kind][x][y] after the z filter: kind 0 value, 1 second difference
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
          const double* row = beta + ((int64_t)xi[a] * n2 + yi[b]) * n3 * n_col + c;
          const double m = row[(int64_t)zi[0] * n_col], z0 = row[(int64_t)zi[1] * n_col], pl = row[(int64_t)zi[2] * n_col];
          zs[0][a][b] = sixth * fmaa(4.0, z0, m + pl);
          zs[1][a][b] = fmaa(-2.0, z0, m + pl);
        }
      double ys[2][2][3];   // [ky kind][kz kind][x]
      for (int kz = 0; kz < 2; ++kz)
        for (int a = 0; a < 3; ++a) {
          const double m = zs[kz][a][0], y0 = zs[kz][a][1], pl = zs[kz][a][2];
          ys[0][kz][a] = sixth * fmaa(4.0, y0, m + pl);
          ys[1][kz][a] = fmaa(-2.0, y0, m + pl);
        }
      for (int ky = 0; ky < 2; ++ky)
        for (int kz = 0; kz < 2; ++kz) {
          const double m = ys[ky][kz][0], x0 = ys[ky][kz][1], pl = ys[ky][kz][2];
          sig[2 * ky + kz] = sixth * fmaa(4.0, x0, m + pl);
          sig[4 + 2 * ky + kz] = fmaa(-2.0, x0, m + pl);
        }
    } else {
      for (int q = 0; q < 8; ++q) sig[q] = 0.0;
    }
    for (int q = 0; q < 8; ++q) {
      const int64_t idx = (p * 8 + q) * o_pad + c;
      if constexpr (OUT == OUT_TABLE_F64) static_cast<double*>(table)[idx] = sig[q];
      else if constexpr (OUT == OUT_TABLE_F32) static_cast<float*>(table)[idx] = (float)sig[q];
      else static_cast<uint16_t*>(table)[idx] = f32_to_bf16_rne((float)sig[q]);
    }
  }
}

// One pp-spline table: the B-spline solve of build_one kept in FP64 in `work`, then the knot filters.
int build_one_pp(const spl_desc* d, const double* vals, void* table, double* work, hipStream_t stream) {
  const int64_t n1 = d->grid[0], n2 = d->grid[1], n3 = d->grid[2], no = d->n_col;
  int rc;
  if ((rc = launch_axis(OUT_F64_WORK, vals, work, 1, (int)n1, n2 * n3 * no, 0, stream))) return rc;
  if ((rc = launch_axis(OUT_F64_WORK, work, work, n1, (int)n2, n3 * no, 0, stream))) return rc;
  if ((rc = launch_axis(OUT_F64_WORK, work, work, n1 * n2, (int)n3, no, 0, stream))) return rc;
  const int64_t total = n1 * n2 * n3 * d->o_pad;
  const dim3 grid((unsigned)((total + 255) / 256 < 65536 ? (total + 255) / 256 : 65536));
  if (d->dtype == SPL_F64)
    hipLaunchKernelGGL(k_pp_sigma<OUT_TABLE_F64>, grid, dim3(256), 0, stream, work, table, (int)n1, (int)n2,
                       (int)n3, d->n_col, d->o_pad);
  else if (d->dtype == SPL_F32)
    hipLaunchKernelGGL(k_pp_sigma<OUT_TABLE_F32>, grid, dim3(256), 0, stream, work, table, (int)n1, (int)n2,
                       (int)n3, d->n_col, d->o_pad);
  else
    hipLaunchKernelGGL(k_pp_sigma<OUT_TABLE_BF16>, grid, dim3(256), 0, stream, work, table, (int)n1, (int)n2,
                       (int)n3, d->n_col, d->o_pad);
  return hip_fail(hipGetLastError(), "pp-spline table launch");
}

// One Lagrange table: grid values [N1][N2][N3][n_col] cast into the padded table.
int cast_one(const spl_desc* d, const double* vals, void* table, hipStream_t stream) {
  const int64_t rows = (int64_t)d->grid[0] * d->grid[1] * d->grid[2];
  const int64_t total = rows * d->o_pad;
  const dim3 grid((unsigned)((total + 255) / 256 < 65536 ? (total + 255) / 256 : 65536));
  if (d->dtype == SPL_F64)
    hipLaunchKernelGGL(k_cast_table<OUT_TABLE_F64>, grid, dim3(256), 0, stream, vals, table, rows, d->n_col, d->o_pad);
  else if (d->dtype == SPL_F32)
    hipLaunchKernelGGL(k_cast_table<OUT_TABLE_F32>, grid, dim3(256), 0, stream, vals, table, rows, d->n_col, d->o_pad);
  else
    hipLaunchKernelGGL(k_cast_table<OUT_TABLE_BF16>, grid, dim3(256), 0, stream, vals, table, rows, d->n_col,
                       d->o_pad);
  return hip_fail(hipGetLastError(), "table cast launch");
}

}  // namespace pws

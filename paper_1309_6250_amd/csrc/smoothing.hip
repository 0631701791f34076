// spline_build_smoothing: Fourier-matched (smoothing) B-spline coefficients (App. A, "Smoothing
// B-spline coefficients", Eq. b-splinecoefficients).
//
//   beta(r_lmn) = sum_G (c_G / gamma_G) exp(i G . r_lmn),   r_lmn = a (l/N1, m/N2, n/N3),
//
// gamma_G being the Fourier transform of one tensor-product basis function: per axis m, with the
// phase per grid step theta_m = G . a_m / N_m = 2 pi n_m / N_m, the paper's C = 3/2 basis gives
// (3/2) sinc^4(theta/2); the standard normalization used here gives sinc^4(theta/2), and gamma is
// the product over the three axes.  Dividing by gamma makes the spline's fundamental Fourier
// components equal c_G.  The other tables of a descriptor are the smoothing splines of the
// periodic parts of the gradient, coefficients i (k+G)_c c_G (separate gradients), and of the
// Laplacian, -|k+G|^2 c_G (k = 0 for real orbitals).
//
// Steps on the device: zero a complex grid [N1][N2][N3][n_orb]; scatter c_G / gamma_G into the
// bins (n mod N); inverse DFT along each axis in turn (one line per thread, staged in LDS, direct
// summation with exact twiddle tables, O(N^2) per line: the build is a one-time cost); the last
// axis writes the real part (real orbitals) or both parts (Bloch orbitals: columns 2o, 2o+1)
// into the padded table in the storage dtype.
#include <math.h>

#include "common.hpp"

namespace pws {

typedef double c2v __attribute__((ext_vector_type(2)));   // (re, im)

__device__ __forceinline__ double sinc4_half(double theta) {
  if (theta == 0.0) return 1.0;
  const double h = 0.5 * theta;
  const double s = sin(h) / h;
  const double s2 = s * s;
  return s2 * s2;
}

struct Kvec {
  double k[3];
};

enum { COMP_VALUE = 0, COMP_LAP = 4 };   // 1, 2, 3: Cartesian gradient component 0, 1, 2

// grid[bin(n)][o] += coef[o][g] * scale(g): scale = 1 / gamma_G, times i (k+G)_c for a gradient
// component c, or -|k+G|^2 for the Laplacian.
// One workgroup per tile of 32 planewaves x 32 orbitals: the coefficients are read along g
// (coef is [o][g]) into LDS, each planewave's scale, wave vector and bin are formed once, and the
// grid is updated along o, so both the reads and the atomic adds are contiguous.
constexpr int SCAT_T = 32;

__global__ __launch_bounds__(256) void k_scatter_coef(const int32_t* miller, const c2v* coef, int64_t n_g,
                                                      int32_t n_orb, Geom geo, int32_t comp, Kvec kv, c2v* grid) {
  __shared__ c2v tile[SCAT_T][SCAT_T + 1];           // [o][g], padded against bank conflicts
  __shared__ double s_scale[SCAT_T], s_mul[SCAT_T];  // per planewave: 1/gamma, and the factor of comp
  __shared__ int64_t s_bin[SCAT_T];
  const int64_t g0 = (int64_t)blockIdx.x * SCAT_T;
  const int o0 = (int)blockIdx.y * SCAT_T;
  const int t = (int)threadIdx.x;
  const double two_pi = 6.283185307179586476925286766559;
  for (int e = t; e < SCAT_T * SCAT_T; e += 256) {
    const int oo = e / SCAT_T, gg = e % SCAT_T;
    const int64_t g = g0 + gg;
    const int o = o0 + oo;
    tile[oo][gg] = (g < n_g && o < n_orb) ? coef[(int64_t)o * n_g + g] : c2v{0.0, 0.0};
  }
  if (t < SCAT_T && g0 + t < n_g) {
    const int64_t g = g0 + t;
    const int n0 = miller[3 * g], n1 = miller[3 * g + 1], n2 = miller[3 * g + 2];
    s_scale[t] = 1.0 / (sinc4_half(two_pi * n0 / geo.n[0]) * sinc4_half(two_pi * n1 / geo.n[1]) *
                        sinc4_half(two_pi * n2 / geo.n[2]));
    double q[3], qsq = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      // k + G with G = 2 pi (lattice^-1) n, and lattice^-1 = ainv^T
      q[c] = kv.k[c] + two_pi * fmaa(geo.ainv[6 + c], (double)n2, fmaa(geo.ainv[3 + c], (double)n1, geo.ainv[c] * n0));
      qsq = fmaa(q[c], q[c], qsq);
    }
    // value: 1; Laplacian: -|k+G|^2 (real); gradient component c: i q_c (applied below)
    s_mul[t] = comp == COMP_LAP ? -qsq : (comp == COMP_VALUE ? 1.0 : q[comp - 1]);
    const int b0 = ((n0 % geo.n[0]) + geo.n[0]) % geo.n[0];
    const int b1 = ((n1 % geo.n[1]) + geo.n[1]) % geo.n[1];
    const int b2 = ((n2 % geo.n[2]) + geo.n[2]) % geo.n[2];
    s_bin[t] = ((int64_t)b0 * geo.n[1] + b1) * geo.n[2] + b2;
  }
  __syncthreads();
  for (int e = t; e < SCAT_T * SCAT_T; e += 256) {
    const int gg = e / SCAT_T, oo = e % SCAT_T;
    const int64_t g = g0 + gg;
    const int o = o0 + oo;
    if (g >= n_g || o >= n_orb) continue;
    const c2v c = tile[oo][gg];
    double re = c.x * s_scale[gg], im = c.y * s_scale[gg];
    if (comp == COMP_LAP) {
      re *= s_mul[gg];
      im *= s_mul[gg];
    } else if (comp != COMP_VALUE) {
      const double qc = s_mul[gg];              // i q_c (re + i im) = -q_c im + i q_c re
      const double tr = re;
      re = -qc * im;
      im = qc * tr;
    }
    double* dst = reinterpret_cast<double*>(grid + s_bin[gg] * n_orb + o);
    unsafeAtomicAdd(dst, re);                    // planewaves sharing a bin (too coarse a grid) add up
    unsafeAtomicAdd(dst + 1, im);
  }
}

struct DftArgs {
  c2v* data;             // complex grid viewed as [outer][n][inner]
  void* table;           // final axis: padded table of the storage dtype
  const double* cs;      // cos(2 pi k / n), k = 0 .. n-1
  const double* sn;      // sin(2 pi k / n)
  int64_t n_lines;
  int64_t inner;
  int32_t n;
  int32_t o_pad;
  int32_t bloch;         // final axis: store (re, im) into columns (2o, 2o+1) instead of re into o
  // lines whose samples are all zero, skipped (they stay zero): line (outer, in) holds a nonzero
  // sample only if mask[in / mask_div] != 0; NULL: every line is computed
  const int32_t* mask;
  int64_t mask_div;
  // along the axis, samples j with kb < j < n - kb are zero (kb = band[axis], the largest |Miller
  // index| on that axis): steps over such samples only are skipped.  NULL: none skipped
  const int32_t* band;
  int32_t axis;
};

__device__ __forceinline__ bool line_live(const DftArgs& a, int64_t line) {
  if (line >= a.n_lines) return false;
  return !a.mask || a.mask[(line % a.inner) / a.mask_div] != 0;
}

// Zero the grid rows every stage may read: only samples with b2 inside the axis-2 band are ever
// loaded (stage 3 along axis 2 loads no other; stages 1 and 2 load only lines in occupied columns
// and planes, which lie inside that band).  One workgroup per (b0, b1): the one or two contiguous
// runs of b2 = 0 .. kb and n3 - kb .. n3 - 1, all orbitals.
__global__ __launch_bounds__(256) void k_czero_band(c2v* grid, int32_t n3, int64_t n_orb, const int32_t* band) {
  const int kb = band[2];
  const int64_t col = blockIdx.x;                        // b0 n2 + b1
  c2v* base = grid + col * n3 * n_orb;
  const bool all = 2 * kb + 1 >= n3;
  const int64_t len0 = (all ? n3 : kb + 1) * n_orb;
  for (int64_t i = threadIdx.x; i < len0; i += blockDim.x) base[i] = c2v{0.0, 0.0};
  if (all) return;
  c2v* hi = base + (int64_t)(n3 - kb) * n_orb;
  for (int64_t i = threadIdx.x; i < (int64_t)kb * n_orb; i += blockDim.x) hi[i] = c2v{0.0, 0.0};
}

__global__ __launch_bounds__(256) void k_mask_zero(int32_t* m, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    m[i] = 0;
}

// Which lines of the first two DFT stages can hold nonzero samples: before the first stage (along
// axis 0) the grid is nonzero only in the columns (b1, b2) of the planewaves' Fourier bins, before
// the second (along axis 1) only in their planes b2.
// Also the band of each axis: the largest |Miller index| along it.
__global__ __launch_bounds__(256) void k_line_masks(const int32_t* miller, int64_t n_g, Geom geo, int32_t* col12,
                                                    int32_t* plane2, int32_t* band) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_g) return;
  const int b1 = ((miller[3 * g + 1] % geo.n[1]) + geo.n[1]) % geo.n[1];
  const int b2 = ((miller[3 * g + 2] % geo.n[2]) + geo.n[2]) % geo.n[2];
  col12[(int64_t)b1 * geo.n[2] + b2] = 1;
  plane2[b2] = 1;
#pragma unroll
  for (int c = 0; c < 3; ++c) atomicMax(band + c, abs(miller[3 * g + c]));
}

enum { DFT_INPLACE = 0, DFT_TABLE_F64 = 1, DFT_TABLE_F32 = 2, DFT_TABLE_BF16 = 3 };

__device__ __forceinline__ uint16_t f32_to_bf16_rne_s(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// y_k = sum_j x_j exp(+2 pi i j k / n) along the middle axis, one line per thread.
template <int OUT>
__global__ __launch_bounds__(256) void k_idft_axis(DftArgs a) {
  extern __shared__ double lds_raw[];
  const int tile = blockDim.x;
  const int tid = threadIdx.x;
  const int n = a.n;
  double* tw_c = lds_raw;                 // [n]
  double* tw_s = lds_raw + n;             // [n]
  c2v* x = reinterpret_cast<c2v*>(lds_raw + 2 * n) + tid;   // [n][tile]
  for (int k = tid; k < n; k += tile) {
    tw_c[k] = a.cs[k];
    tw_s[k] = a.sn[k];
  }
  __syncthreads();                        // every thread of the block reaches this barrier
  const int64_t line = (int64_t)blockIdx.x * tile + tid;
  if (!line_live(a, line)) return;
  const int64_t outer = line / a.inner;
  const int64_t in = line - outer * a.inner;
  const int64_t base = outer * (int64_t)n * a.inner + in;
  const int kb = a.band ? min(a.band[a.axis], n) : n;
  for (int j = 0; j < n; ++j)                       // samples outside the band are zero, not loaded
    x[j * tile] = (j > kb && j < n - kb) ? c2v{0.0, 0.0} : a.data[base + (int64_t)j * a.inner];
  for (int k = 0; k < n; ++k) {
    double re = 0.0, im = 0.0;
    int idx = 0;                          // (j k) mod n
    for (int j = 0; j < n; ++j) {
      if (j > kb && j < n - kb) {         // zero samples: jump to the upper end of the band
        idx = (int)(((int64_t)k * (n - kb)) % n);
        j = n - kb - 1;
        continue;
      }
      const c2v v = x[j * tile];
      const double c = tw_c[idx], s = tw_s[idx];
      re = fmaa(v.x, c, fmaa(-v.y, s, re));
      im = fmaa(v.x, s, fmaa(v.y, c, im));
      idx += k;
      if (idx >= n) idx -= n;
    }
    if constexpr (OUT == DFT_INPLACE) {
      a.data[base + (int64_t)k * a.inner] = c2v{re, im};
    } else {
      const int64_t row = (outer * (int64_t)n + k) * a.o_pad;      // inner == n_orb here
      const int64_t t = a.bloch ? row + 2 * in : row + in;
      if constexpr (OUT == DFT_TABLE_F64) {
        static_cast<double*>(a.table)[t] = re;
        if (a.bloch) static_cast<double*>(a.table)[t + 1] = im;
      } else if constexpr (OUT == DFT_TABLE_F32) {
        static_cast<float*>(a.table)[t] = (float)re;
        if (a.bloch) static_cast<float*>(a.table)[t + 1] = (float)im;
      } else {
        static_cast<uint16_t*>(a.table)[t] = f32_to_bf16_rne_s((float)re);
        if (a.bloch) static_cast<uint16_t*>(a.table)[t + 1] = f32_to_bf16_rne_s((float)im);
      }
    }
  }
}

// The same stage as a matrix product on the FP64 matrix cores: along the axis, Y = W X with
// W[k][j] = exp(+2 pi i j k / n) and X the n samples of each line.  One workgroup owns 16 whole
// lines (so the in-place update is safe): it stages their samples in LDS, then its waves form
// alternate tiles of 16 outputs x 16 lines with 16x16x4 steps over j, four real products per step
// (complex multiply).
typedef double f64x4_s __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f64x4_s mfma64(double a, double b, f64x4_s c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// waves per workgroup sharing the staged lines: 3 splits the output tiles of 48, 96, 144 and 192
// points evenly (three waves 6.8 ms on the MgO-like cell, six 6.7, two 7.8, one 10.4)
constexpr int DFT_WAVES = 3;

template <int OUT>
__global__ __launch_bounds__(64 * DFT_WAVES) void k_idft_mfma(DftArgs a) {
  extern __shared__ double lds_raw[];
  const int n = a.n;
  const int n_pad = (n + 3) & ~3;
  double* tw_c = lds_raw;                 // [n]
  double* tw_s = lds_raw + n;             // [n]
  double* xr = lds_raw + 2 * n;           // [n_pad][16] real parts of the 16 lines
  double* xi = xr + 16 * n_pad;           // imaginary parts
  const int tid = (int)threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int grp = lane >> 4, col = lane & 15;
  const int64_t line0 = (int64_t)blockIdx.x * 16;
  // if none of the workgroup's 16 lines can be nonzero, they stay zero (every wave decides alike)
  if (!__any(line_live(a, line0 + col))) return;
  for (int k = tid; k < n; k += 64 * DFT_WAVES) {
    tw_c[k] = a.cs[k];
    tw_s[k] = a.sn[k];
  }
  const int kb = a.band ? min(a.band[a.axis], n) : n;
  for (int e = tid; e < 16 * n_pad; e += 64 * DFT_WAVES) {
    const int j = e >> 4, c = e & 15;
    const int64_t line = line0 + c;
    c2v v{0.0, 0.0};
    if (j < n && line < a.n_lines && !(j > kb && j < n - kb)) {   // samples outside the band are zero
      const int64_t outer = line / a.inner;
      v = a.data[outer * (int64_t)n * a.inner + (line - outer * a.inner) + (int64_t)j * a.inner];
    }
    xr[e] = v.x;
    xi[e] = v.y;
  }
  __syncthreads();
  // this lane's output line (column of the result tile)
  const int64_t line = line0 + col;
  const bool line_ok = line < a.n_lines;
  const int64_t outer = line_ok ? line / a.inner : 0;
  const int64_t in = line_ok ? line - outer * a.inner : 0;
  const int64_t base = outer * (int64_t)n * a.inner + in;
  // the last stage of a real table stores the real part only: the imaginary products are skipped
  const bool need_im = OUT == DFT_INPLACE || a.bloch;
  // every sample is in LDS before the barrier above, so the waves may overwrite the lines in place
  for (int k0 = 16 * wave; k0 < n; k0 += 16 * DFT_WAVES) {
    f64x4_s acc_r = {0.0, 0.0, 0.0, 0.0}, acc_i = {0.0, 0.0, 0.0, 0.0};
    const int kk = k0 + col;              // A row: output index (past n: any finite value, not written)
    // twiddle index (kk j) mod n of this lane's sample j = j0 + grp, advanced by 4 kk mod n per step
    const int step = (int)((4 * (int64_t)kk) % n);
    int idx = (int)(((int64_t)kk * grp) % n);
    for (int j0 = 0; j0 < n_pad; j0 += 4, idx = idx + step >= n ? idx + step - n : idx + step) {
      if (j0 > kb && j0 + 3 < n - kb) continue;   // four zero samples
      const int j = j0 + grp;             // A column / B row: sample index (past n: X is zero)
      const double c = tw_c[idx], sn = tw_s[idx];
      const double br = xr[j * 16 + col], bi = xi[j * 16 + col];
      acc_r = mfma64(c, br, acc_r);
      acc_r = mfma64(-sn, bi, acc_r);
      if (need_im) {
        acc_i = mfma64(sn, br, acc_i);
        acc_i = mfma64(c, bi, acc_i);
      }
    }
    if (!line_ok) continue;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int k = k0 + grp + 4 * e;     // FP64 result layout: row grp + 4 e, column col
      if (k >= n) continue;
      const double re = acc_r[e], im = acc_i[e];
      if constexpr (OUT == DFT_INPLACE) {
        a.data[base + (int64_t)k * a.inner] = c2v{re, im};
      } else {
        const int64_t row = (outer * (int64_t)n + k) * a.o_pad;      // inner == n_orb here
        const int64_t t = a.bloch ? row + 2 * in : row + in;
        if constexpr (OUT == DFT_TABLE_F64) {
          static_cast<double*>(a.table)[t] = re;
          if (a.bloch) static_cast<double*>(a.table)[t + 1] = im;
        } else if constexpr (OUT == DFT_TABLE_F32) {
          static_cast<float*>(a.table)[t] = (float)re;
          if (a.bloch) static_cast<float*>(a.table)[t + 1] = (float)im;
        } else {
          static_cast<uint16_t*>(a.table)[t] = f32_to_bf16_rne_s((float)re);
          if (a.bloch) static_cast<uint16_t*>(a.table)[t + 1] = f32_to_bf16_rne_s((float)im);
        }
      }
    }
  }
}

template <typename TS>
__global__ __launch_bounds__(256) void k_zero_pad_s(TS* table, int64_t n_rows, int32_t n_col, int32_t o_pad) {
  const int32_t width = o_pad - n_col;
  const int64_t total = n_rows * width;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / width;
    table[r * o_pad + n_col + (i - r * width)] = TS(0);
  }
}

static int dft_tile(int n) {
  int tile = 256;
  while (tile > 4 && (int64_t)tile * n * 16 + 16 * (int64_t)n > 65536) tile >>= 1;
  return tile;
}

// One inverse-DFT stage along the middle axis of [outer][n][inner] (twiddles in the workspace).
static int launch_idft(int out, c2v* data, void* table, const double* cs, const double* sn, int64_t outer, int n,
                       int64_t inner, int o_pad, int bloch, const int32_t* mask, int64_t mask_div,
                       const int32_t* band, int axis, hipStream_t stream) {
  DftArgs a;
  a.mask = mask;
  a.mask_div = mask_div;
  a.band = band;
  a.axis = axis;
  a.data = data;
  a.table = table;
  a.cs = cs;
  a.sn = sn;
  a.n_lines = outer * inner;
  a.inner = inner;
  a.n = n;
  a.o_pad = o_pad;
  a.bloch = bloch;
  if (n <= 192) {
    // matrix-core form: 16 lines per workgroup, staged samples and twiddles in LDS (at most 52 KB)
    const size_t shm = (size_t)(2 * n + 32 * ((n + 3) & ~3)) * sizeof(double);
    const dim3 g((unsigned)((a.n_lines + 15) / 16)), b(64 * DFT_WAVES);
    switch (out) {
      case DFT_INPLACE: hipLaunchKernelGGL(k_idft_mfma<DFT_INPLACE>, g, b, shm, stream, a); break;
      case DFT_TABLE_F64: hipLaunchKernelGGL(k_idft_mfma<DFT_TABLE_F64>, g, b, shm, stream, a); break;
      case DFT_TABLE_F32: hipLaunchKernelGGL(k_idft_mfma<DFT_TABLE_F32>, g, b, shm, stream, a); break;
      default: hipLaunchKernelGGL(k_idft_mfma<DFT_TABLE_BF16>, g, b, shm, stream, a); break;
    }
    return hip_fail(hipGetLastError(), "inverse DFT launch");
  }
  const int tile = dft_tile(n);
  const size_t shmem = (size_t)tile * n * 16 + (size_t)n * 16;
  const dim3 grid((unsigned)((a.n_lines + tile - 1) / tile));
  switch (out) {
    case DFT_INPLACE: hipLaunchKernelGGL(k_idft_axis<DFT_INPLACE>, grid, dim3(tile), shmem, stream, a); break;
    case DFT_TABLE_F64: hipLaunchKernelGGL(k_idft_axis<DFT_TABLE_F64>, grid, dim3(tile), shmem, stream, a); break;
    case DFT_TABLE_F32: hipLaunchKernelGGL(k_idft_axis<DFT_TABLE_F32>, grid, dim3(tile), shmem, stream, a); break;
    default: hipLaunchKernelGGL(k_idft_axis<DFT_TABLE_BF16>, grid, dim3(tile), shmem, stream, a); break;
  }
  return hip_fail(hipGetLastError(), "inverse DFT launch");
}

int build_smoothing_one(const spl_desc* d, int64_t n_g, const int32_t* miller, const double* coef, int comp,
                        void* table, void* work, const double* twiddles, const int32_t* col12,
                        const int32_t* plane2, const int32_t* band, hipStream_t stream) {
  const int64_t n1 = d->grid[0], n2 = d->grid[1], n3 = d->grid[2], no = d->n_orb;
  c2v* grid = static_cast<c2v*>(work);
  int rc;
  hipLaunchKernelGGL(k_czero_band, dim3((unsigned)(n1 * n2)), dim3(256), 0, stream, grid, (int32_t)n3, no, band);
  if ((rc = hip_fail(hipGetLastError(), "zero fill launch"))) return rc;
  const Geom geo = make_geom(d);
  Kvec kv;
  for (int c = 0; c < 3; ++c) kv.k[c] = d->kvec[c];
  if (n_g > 0) {
    const dim3 sg((unsigned)((n_g + SCAT_T - 1) / SCAT_T), (unsigned)((no + SCAT_T - 1) / SCAT_T));
    hipLaunchKernelGGL(k_scatter_coef, sg, dim3(256), 0, stream, miller, reinterpret_cast<const c2v*>(coef), n_g,
                       (int32_t)no, geo, (int32_t)comp, kv, grid);
    if ((rc = hip_fail(hipGetLastError(), "coefficient scatter launch"))) return rc;
  }
  // twiddles: [axis][cos n | sin n] packed one axis after the other
  const double* tw0 = twiddles;
  const double* tw1 = tw0 + 2 * n1;
  const double* tw2 = tw1 + 2 * n2;
  // stage 1 lines (b1, b2, o) and stage 2 lines (x, b2, o): only those of occupied columns / planes
  if ((rc = launch_idft(DFT_INPLACE, grid, nullptr, tw0, tw0 + n1, 1, (int)n1, n2 * n3 * no, 0, 0, col12, no,
                        band, 0, stream)))
    return rc;
  if ((rc = launch_idft(DFT_INPLACE, grid, nullptr, tw1, tw1 + n2, n1, (int)n2, n3 * no, 0, 0, plane2, no, band, 1,
                        stream)))
    return rc;
  const int out = d->dtype == SPL_F64 ? DFT_TABLE_F64 : d->dtype == SPL_F32 ? DFT_TABLE_F32 : DFT_TABLE_BF16;
  if ((rc = launch_idft(out, grid, table, tw2, tw2 + n3, n1 * n2, (int)n3, no, d->o_pad, d->bloch, nullptr, 1, band,
                        2, stream)))
    return rc;
  if (d->o_pad > d->n_col) {
    const int64_t rows = n1 * n2 * n3;
    const int64_t total = rows * (d->o_pad - d->n_col);
    const dim3 g((unsigned)std::min<int64_t>((total + 255) / 256, 65536));
    if (d->dtype == SPL_F64)
      hipLaunchKernelGGL(k_zero_pad_s<double>, g, dim3(256), 0, stream, (double*)table, rows, d->n_col, d->o_pad);
    else if (d->dtype == SPL_F32)
      hipLaunchKernelGGL(k_zero_pad_s<float>, g, dim3(256), 0, stream, (float*)table, rows, d->n_col, d->o_pad);
    else
      hipLaunchKernelGGL(k_zero_pad_s<uint16_t>, g, dim3(256), 0, stream, (uint16_t*)table, rows, d->n_col, d->o_pad);
    if ((rc = hip_fail(hipGetLastError(), "zero padding launch"))) return rc;
  }
  return SPL_OK;
}

// Twiddle tables of the three axes, packed [cos(2 pi k / N1) | sin(..) | cos(.. N2) | sin | cos(.. N3) | sin].
__global__ void k_twiddles(double* tw, int32_t n0, int32_t n1, int32_t n2) {
  const int k = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  const double two_pi = 6.283185307179586476925286766559;
  int n = n0, base = 0, kk = k;
  if (kk >= n0) { kk -= n0; base = 2 * n0; n = n1;
    if (kk >= n1) { kk -= n1; base = 2 * (n0 + n1); n = n2; if (kk >= n2) return; } }
  const double ang = two_pi * kk / n;
  tw[base + kk] = cos(ang);
  tw[base + n + kk] = sin(ang);
}

// workspace: the complex grid, 256-byte aligned twiddles, then the two line masks and the bands
int64_t smoothing_work_bytes(const spl_desc* d) {
  const int64_t cells = (int64_t)d->grid[0] * d->grid[1] * d->grid[2] * d->n_orb;
  const int64_t tw = 16 * (int64_t)(d->grid[0] + d->grid[1] + d->grid[2]);
  return ((cells * 16 + 255) & ~int64_t(255)) + ((tw + 255) & ~int64_t(255)) +
         4 * ((int64_t)d->grid[1] * d->grid[2] + d->grid[2] + 3);
}

int build_smoothing(const spl_desc* d, int64_t n_g, const int32_t* miller, const double* coef, void* table,
                    void* work, hipStream_t stream) {
  const int64_t cells = (int64_t)d->grid[0] * d->grid[1] * d->grid[2] * d->n_orb;
  double* tw = reinterpret_cast<double*>(static_cast<char*>(work) + ((cells * 16 + 255) & ~int64_t(255)));
  const int nt = d->grid[0] + d->grid[1] + d->grid[2];
  hipLaunchKernelGGL(k_twiddles, dim3((nt + 255) / 256), dim3(256), 0, stream, tw, d->grid[0], d->grid[1], d->grid[2]);
  int rc = hip_fail(hipGetLastError(), "twiddle launch");
  if (rc) return rc;
  // line masks after the twiddles (the same for every table: they depend on the planewaves only)
  int32_t* col12 = reinterpret_cast<int32_t*>(reinterpret_cast<char*>(tw) + ((16 * (int64_t)nt + 255) & ~int64_t(255)));
  const int64_t n12 = (int64_t)d->grid[1] * d->grid[2];
  int32_t* plane2 = col12 + n12;
  int32_t* band = plane2 + d->grid[2];
  const int64_t n_mask = n12 + d->grid[2] + 3;
  hipLaunchKernelGGL(k_mask_zero, dim3((unsigned)std::min<int64_t>((n_mask + 255) / 256, 4096)), dim3(256), 0, stream,
                     col12, n_mask);
  if ((rc = hip_fail(hipGetLastError(), "mask clear launch"))) return rc;
  if (n_g > 0) {
    hipLaunchKernelGGL(k_line_masks, dim3((unsigned)((n_g + 255) / 256)), dim3(256), 0, stream, miller, n_g,
                       make_geom(d), col12, plane2, band);
    if ((rc = hip_fail(hipGetLastError(), "line mask launch"))) return rc;
  }
  // tables in order: orbital, gradient components x, y, z (sep_grad), Laplacian (has_lap)
  for (int t = 0; t < d->n_tables; ++t) {
    const int comp = t == 0 ? COMP_VALUE : (d->sep_grad && t <= 3 ? t : COMP_LAP);
    char* dst = static_cast<char*>(table) + t * d->table_elems * d->elem_bytes;
    if ((rc = build_smoothing_one(d, n_g, miller, coef, comp, dst, work, tw, col12, plane2, band, stream))) return rc;
  }
  return SPL_OK;
}

}  // namespace pws

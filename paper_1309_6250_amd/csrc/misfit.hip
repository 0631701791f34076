// The two terms of the least-squares fit of coefficients to orbital samples.
//
// spline_misfit, the data term.
// For n outputs y (values or Laplacians of the spline at the fit points) and their targets t:
//     loss += w sum_i (y_i - t_i)^2,        g_i = 2 w (y_i - t_i),
// g being the upstream gradient that spline_eval_vgl_backward turns into the gradient of the
// loss with respect to the coefficients.  One pass over y and t, HBM-bound.
//
// The sum is formed in FP64 and in a fixed order: MISFIT_BLOCKS workgroups each own the same
// grid-strided elements on every call and reduce them in a fixed tree in LDS; one workgroup
// then adds the partial sums in a fixed tree and the result to *loss.  So the loss is
// reproducible bit for bit, like the deterministic adjoint it feeds.
#include <algorithm>
#include <cmath>

#include "common.hpp"
#include "update.hpp"

namespace pws {

constexpr int MISFIT_BLOCKS = 1024;
constexpr int MISFIT_THREADS = 256;

template <typename T>
__global__ __launch_bounds__(MISFIT_THREADS) void k_misfit(int64_t n, const T* y, const T* t, T two_w, T* g,
                                                           double* partial) {
  __shared__ double red[MISFIT_THREADS];
  const int64_t stride = (int64_t)MISFIT_BLOCKS * MISFIT_THREADS;
  double s = 0.0;
  int64_t i = (int64_t)blockIdx.x * MISFIT_THREADS + threadIdx.x;
  // four independent loads in flight per thread
  for (; i + 3 * stride < n; i += 4 * stride) {
    T r[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) r[u] = y[i + u * stride] - t[i + u * stride];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      s += (double)r[u] * (double)r[u];
      g[i + u * stride] = two_w * r[u];
    }
  }
  for (; i < n; i += stride) {
    const T r = y[i] - t[i];
    s += (double)r * (double)r;
    g[i] = two_w * r;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = MISFIT_THREADS / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(MISFIT_THREADS) void k_misfit_total(const double* partial, double w, double* loss) {
  __shared__ double red[MISFIT_THREADS];
  double s = 0.0;
  for (int b = threadIdx.x; b < MISFIT_BLOCKS; b += MISFIT_THREADS) s += partial[b];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = MISFIT_THREADS / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss += w * red[0];
}

// spline_smoothness_penalty, the regularizer: with D the periodic second difference along one grid
// axis, for the orbital table beta and its real orbitals o < n_orb,
//     loss  += w sum over axes, grid points and orbitals of (D beta)^2
//     gbeta += 2 w sum over axes of D (D beta)        (D is symmetric under the periodic wrap;
//              D D = the five-point stencil 1 -4 6 -4 1)
// MISFIT_BLOCKS workgroups of four waves take the table rows (grid points) in a fixed stride, each
// wave its own rows, one lane per orbital, in FP64 whatever the storage type: a row's index and its
// periodic neighbours' offsets are worked out once for all of its orbitals.  Each workgroup's sum is
// reduced in LDS and the MISFIT_BLOCKS partial sums like the misfit's.
template <typename TS> struct Coef;
template <> struct Coef<double> {
  __device__ __forceinline__ static double at(const double* p) { return *p; }
};
template <> struct Coef<float> {
  __device__ __forceinline__ static double at(const float* p) { return (double)*p; }
};
template <> struct Coef<uint16_t> {   // BF16 bits
  __device__ __forceinline__ static double at(const uint16_t* p) { return (double)__uint_as_float((uint32_t)*p << 16); }
};

constexpr int PENALTY_THREADS = 256;

template <typename TS, typename GO>
__global__ __launch_bounds__(PENALTY_THREADS) void k_penalty(Geom g, const TS* beta, int32_t n_orb, double w,
                                                             GO* gbeta, double* partial) {
  __shared__ double red[PENALTY_THREADS];
  constexpr int WAVES = PENALTY_THREADS / 64;
  const int wave = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
  const int64_t n_rows = (int64_t)g.n[0] * g.n[1] * g.n[2];
  const int64_t step[3] = {g.s0, g.s1, g.o_pad};
  double s = 0.0;
  for (int64_t r = blockIdx.x + (int64_t)wave * MISFIT_BLOCKS; r < n_rows; r += (int64_t)WAVES * MISFIT_BLOCKS) {
    const int idx[3] = {(int)(r / ((int64_t)g.n[1] * g.n[2])), (int)((r / g.n[2]) % g.n[1]), (int)(r % g.n[2])};
    const int64_t row = idx[0] * g.s0 + idx[1] * g.s1 + idx[2] * (int64_t)g.o_pad;
    int64_t nb[3][4];                      // offsets of the neighbours at -2, -1, +1, +2 along each axis, periodic
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const int N = g.n[ax];
      const int ks[4] = {-2, -1, 1, 2};
#pragma unroll
      for (int q = 0; q < 4; ++q) nb[ax][q] = (int64_t)((idx[ax] + ks[q] + 2 * N) % N - idx[ax]) * step[ax];
    }
#pragma unroll 2
    for (int o = lane; o < n_orb; o += 64) {
      const int64_t base = row + o;
      const double b0 = Coef<TS>::at(beta + base);
      double grad = 0.0;
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) {
        const double m2 = Coef<TS>::at(beta + base + nb[ax][0]), m1 = Coef<TS>::at(beta + base + nb[ax][1]);
        const double p1 = Coef<TS>::at(beta + base + nb[ax][2]), p2 = Coef<TS>::at(beta + base + nb[ax][3]);
        const double d2 = m1 - 2.0 * b0 + p1;
        s += d2 * d2;
        grad += (m2 + p2) - 4.0 * (m1 + p1) + 6.0 * b0;
      }
      GO* gp = gbeta + base;
      *gp = (GO)((double)*gp + 2.0 * w * grad);
    }
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = PENALTY_THREADS / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// spline_adam_step: one Adam update of n stored coefficients from their gradient and moments, in
// the precision of the moments (FP64 for FP64 tables, else FP32; BF16 coefficients are widened and
// rounded back to nearest even).  Element-wise, so every element's bits are fixed.
template <typename TS> struct Stored1;
template <> struct Stored1<double> {
  __device__ __forceinline__ static double get(const double* p) { return *p; }
  __device__ __forceinline__ static void put(double* p, double x) { *p = x; }
};
template <> struct Stored1<float> {
  __device__ __forceinline__ static float get(const float* p) { return *p; }
  __device__ __forceinline__ static void put(float* p, float x) { *p = x; }
};
template <> struct Stored1<uint16_t> {
  __device__ __forceinline__ static float get(const uint16_t* p) { return __uint_as_float((uint32_t)*p << 16); }
  __device__ __forceinline__ static void put(uint16_t* p, float x) { *p = f32_to_bf16_rne(x); }
};

template <typename TS>
__global__ __launch_bounds__(256) void k_adam(int64_t n, TS* param, const typename Acc<TS>::type* grad,
                                              typename Acc<TS>::type* m, typename Acc<TS>::type* v,
                                              AdamCoef<typename Acc<TS>::type> k) {
  using T = typename Acc<TS>::type;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    T p = Stored1<TS>::get(param + i), mi = m[i], vi = v[i];
    adam_update<T>(k, grad[i], p, mi, vi);
    Stored1<TS>::put(param + i, p);
    m[i] = mi;
    v[i] = vi;
  }
}

}  // namespace pws

using namespace pws;

extern "C" {

int spline_misfit_work_bytes(const spl_desc* d, int64_t n, int64_t* bytes) {
  clear_error();
  int rc = check_desc(d);
  if (rc) return rc;
  if (n < 0 || !bytes) return fail(SPL_EINVAL, "n < 0 or bytes is NULL");
  *bytes = (int64_t)MISFIT_BLOCKS * (int64_t)sizeof(double);
  return SPL_OK;
}

int spline_misfit(const spl_desc* d, int64_t n, const void* y, const void* t, double w, void* g, double* loss,
                  void* work, int64_t work_bytes, void* stream) {
  clear_error();
  int rc = check_desc(d);
  if (rc) return rc;
  if (n < 0) return fail(SPL_EINVAL, "n < 0");
  if (!std::isfinite(w)) return fail(SPL_EINVAL, "weight is not finite");
  if (n == 0) return SPL_OK;
  if (!y || !t || !g || !loss || !work) return fail(SPL_EINVAL, "NULL y, t, g, loss or work");
  if (work_bytes < (int64_t)MISFIT_BLOCKS * (int64_t)sizeof(double))
    return fail(SPL_EINVAL, "work must hold %d bytes", MISFIT_BLOCKS * (int)sizeof(double));
  const size_t es = d->dtype == SPL_F64 ? 8 : 4;
  for (const void* p : {y, t, static_cast<const void*>(g)})
    if ((uintptr_t)p % es) return fail(SPL_EINVAL, "y, t and g must be aligned to their element size");
  if ((uintptr_t)loss % 8 || (uintptr_t)work % 8) return fail(SPL_EINVAL, "loss and work must be 8-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  double* partial = static_cast<double*>(work);
  if (d->dtype == SPL_F64)
    hipLaunchKernelGGL(k_misfit<double>, dim3(MISFIT_BLOCKS), dim3(MISFIT_THREADS), 0, s, n,
                       static_cast<const double*>(y), static_cast<const double*>(t), 2.0 * w,
                       static_cast<double*>(g), partial);
  else
    hipLaunchKernelGGL(k_misfit<float>, dim3(MISFIT_BLOCKS), dim3(MISFIT_THREADS), 0, s, n,
                       static_cast<const float*>(y), static_cast<const float*>(t), (float)(2.0 * w),
                       static_cast<float*>(g), partial);
  if ((rc = hip_fail(hipGetLastError(), "misfit launch"))) return rc;
  hipLaunchKernelGGL(k_misfit_total, dim3(1), dim3(MISFIT_THREADS), 0, s, partial, w, loss);
  return hip_fail(hipGetLastError(), "misfit total launch");
}

int spline_smoothness_penalty(const spl_desc* d, const void* table, double w, void* gtable, double* loss,
                              void* work, int64_t work_bytes, void* stream) {
  clear_error();
  int rc = check_desc(d);
  if (rc) return rc;
  if (d->basis != SPL_BSPLINE || d->sep_grad || d->bloch)
    return fail(SPL_EUNSUPPORTED, "the penalty covers real B-spline tables without separate gradients");
  if (!std::isfinite(w)) return fail(SPL_EINVAL, "weight is not finite");
  if (!table || !gtable || !loss || !work) return fail(SPL_EINVAL, "NULL table, gtable, loss or work");
  if (work_bytes < (int64_t)MISFIT_BLOCKS * (int64_t)sizeof(double))
    return fail(SPL_EINVAL, "work must hold %d bytes", MISFIT_BLOCKS * (int)sizeof(double));
  const size_t gs = d->dtype == SPL_F64 ? 8 : 4;
  if ((uintptr_t)table % (size_t)d->elem_bytes || (uintptr_t)gtable % gs || (uintptr_t)loss % 8 ||
      (uintptr_t)work % 8)
    return fail(SPL_EINVAL, "table, gtable, loss or work misaligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  double* partial = static_cast<double*>(work);
  const Geom g = make_geom(d);
  if (d->dtype == SPL_F64)
    hipLaunchKernelGGL((k_penalty<double, double>), dim3(MISFIT_BLOCKS), dim3(PENALTY_THREADS), 0, s, g,
                       static_cast<const double*>(table), d->n_orb, w, static_cast<double*>(gtable), partial);
  else if (d->dtype == SPL_F32)
    hipLaunchKernelGGL((k_penalty<float, float>), dim3(MISFIT_BLOCKS), dim3(PENALTY_THREADS), 0, s, g,
                       static_cast<const float*>(table), d->n_orb, w, static_cast<float*>(gtable), partial);
  else
    hipLaunchKernelGGL((k_penalty<uint16_t, float>), dim3(MISFIT_BLOCKS), dim3(PENALTY_THREADS), 0, s, g,
                       static_cast<const uint16_t*>(table), d->n_orb, w, static_cast<float*>(gtable), partial);
  if ((rc = hip_fail(hipGetLastError(), "penalty launch"))) return rc;
  hipLaunchKernelGGL(k_misfit_total, dim3(1), dim3(MISFIT_THREADS), 0, s, partial, w, loss);
  return hip_fail(hipGetLastError(), "penalty total launch");
}

int spline_adam_step(int32_t dtype, int64_t n, void* param, const void* grad, void* m, void* v, double lr,
                     double beta1, double beta2, double eps, int32_t step, void* stream) {
  clear_error();
  if (dtype != SPL_F64 && dtype != SPL_F32 && dtype != SPL_BF16) return fail(SPL_EDTYPE, "dtype %d", dtype);
  if (n < 0) return fail(SPL_EINVAL, "n = %lld < 0", (long long)n);
  if (!std::isfinite(lr) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) ||
      !(eps > 0.0 && std::isfinite(eps)) || step < 1)
    return fail(SPL_EINVAL, "lr, beta1, beta2, eps or step out of range");
  if (n == 0) return SPL_OK;
  const uintptr_t ps = dtype == SPL_F64 ? 8 : (dtype == SPL_F32 ? 4 : 2), ms = dtype == SPL_F64 ? 8 : 4;
  if (!param || !grad || !m || !v) return fail(SPL_EINVAL, "NULL param, grad, m or v");
  if ((uintptr_t)param % ps || (uintptr_t)grad % ms || (uintptr_t)m % ms || (uintptr_t)v % ms)
    return fail(SPL_EINVAL, "param, grad, m or v misaligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 8192);
  if (dtype == SPL_F64)
    hipLaunchKernelGGL(k_adam<double>, dim3(grid), dim3(256), 0, s, n, static_cast<double*>(param),
                       static_cast<const double*>(grad), static_cast<double*>(m), static_cast<double*>(v),
                       adam_coef<double>(lr, beta1, beta2, eps, step));
  else if (dtype == SPL_F32)
    hipLaunchKernelGGL(k_adam<float>, dim3(grid), dim3(256), 0, s, n, static_cast<float*>(param),
                       static_cast<const float*>(grad), static_cast<float*>(m), static_cast<float*>(v),
                       adam_coef<float>(lr, beta1, beta2, eps, step));
  else
    hipLaunchKernelGGL(k_adam<uint16_t>, dim3(grid), dim3(256), 0, s, n, static_cast<uint16_t*>(param),
                       static_cast<const float*>(grad), static_cast<float*>(m), static_cast<float*>(v),
                       adam_coef<float>(lr, beta1, beta2, eps, step));
  return hip_fail(hipGetLastError(), "adam launch");
}

}  // extern "C"
